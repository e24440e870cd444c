// Host side of the C ABI declared in include/se.h: argument validation,
// workspace carving and kernel sequencing.  Nothing here computes any part
// of the method; every step runs in the HIP kernels of this directory.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <numeric>
#include <unordered_map>
#include <vector>

#include "se_internal.h"

namespace sefase {

static thread_local char g_err[512] = "";

se_status fail(se_status code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

se_status check_launch(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(SE_EHIP, "%s: %s", what, hipGetErrorString(e));
  return SE_OK;
}

static inline int round4(int v) { return (v + 3) & ~3; }

// Frames and area shape the descriptors are checked against when they are
// uploaded for a loop (blocks without an available sample are marked).
struct AreaShape {
  int H, W, T, M, N;
};

// Copies n_blk descriptors to the device (ld = 0 read as 1); with `shape`,
// marks the blocks that have no available sample (kBlockNoSupport) and
// counts them into *n_deg.
static se_status upload_blocks(const se_block* blocks, int n_blk, DevBlock* dst, hipStream_t s,
                               const AreaShape* shape = nullptr, int* n_deg = nullptr) {
  std::vector<DevBlock> tmp((size_t)n_blk);
  int deg = 0;
  for (int i = 0; i < n_blk; ++i) {
    const se_block& b = blocks[i];
    const bool none = shape && block_without_support(b, shape->H, shape->W, shape->T, shape->M,
                                                     shape->N);
    deg += none;
    tmp[(size_t)i] = DevBlock{b.img, b.y0, b.x0, b.ly, b.lx, b.lh, b.lw,
                              none ? kBlockNoSupport : 0, b.lt, b.ld < 1 ? 1 : b.ld};
  }
  if (n_deg) *n_deg = deg;
  // pageable source: the call returns once the data has been staged
  const hipError_t e = hipMemcpyAsync(dst, tmp.data(), tmp.size() * sizeof(DevBlock),
                                      hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return fail(SE_EHIP, "block upload: %s", hipGetErrorString(e));
  return SE_OK;
}

// Descriptors as the caller wrote them, normalised on the device the way
// upload_blocks writes them (ld = 0 read as 1, the blocks without an
// available sample marked): the upload of the allocation-free entry point
// needs no host staging buffer.
__global__ void k_normalize_blocks(se_block* b, int n, AreaShape sh) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  se_block v = b[i];
  v.geom = block_without_support(v, sh.H, sh.W, sh.T, sh.M, sh.N) ? kBlockNoSupport : 0;
  v.ld = v.ld < 1 ? 1 : v.ld;
  b[i] = v;
}

static se_status upload_blocks_raw(const se_block* blocks, int n_blk, DevBlock* dst,
                                   hipStream_t s, const AreaShape& shape) {
  // pageable source: the call returns once the data has been staged
  const hipError_t e = hipMemcpyAsync(dst, blocks, (size_t)n_blk * sizeof(se_block),
                                      hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return fail(SE_EHIP, "block upload: %s", hipGetErrorString(e));
  hipLaunchKernelGGL(k_normalize_blocks, dim3((n_blk + 255) / 256), dim3(256), 0, s, dst, n_blk,
                     shape);
  return check_launch("normalize_blocks");
}

// The count of blocks without an available sample (host side).
static int count_without_support(const se_block* blocks, int n_blk, const AreaShape& sh) {
  int n = 0;
  for (int i = 0; i < n_blk; ++i) n += block_without_support(blocks[i], sh.H, sh.W, sh.T, sh.M, sh.N);
  return n;
}

// SE_ENUMERIC for a call that finished its other blocks but found n_deg
// blocks with nothing to extrapolate from.
static se_status degenerate_status(int n_deg) {
  if (n_deg == 0) return SE_OK;
  return fail(SE_ENUMERIC, "%d block(s) have no available sample in their area: sel = -1, loss "
              "left unchanged", n_deg);
}

// ---------------------------------------------------------------------------
// Workspace of the allocation-free entry point: a static device array, one
// copy per GPU (each device that loads the library's code object holds it
// until the process ends).  In host code `scratch` names a host-side stand-in
// only; kernels and copies get the device address that hipGetSymbolAddress
// returns, looked up once per device with that device current.
static __device__ __align__(256) unsigned char scratch[SE_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_dev[kMaxDevices];

// Device address of `scratch` on the device `stream` belongs to (the current
// device for the null stream).
static se_status static_scratch(hipStream_t s, void** out) {
  int cur = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return fail(SE_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
  int dev = cur;
  if (s && (e = hipStreamGetDevice(s, &dev)) != hipSuccess)
    return fail(SE_EHIP, "hipStreamGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(SE_EINVAL, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    if (dev != cur && (e = hipSetDevice(dev)) != hipSuccess)
      return fail(SE_EHIP, "hipSetDevice(%d): %s", dev, hipGetErrorString(e));
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (dev != cur) hipSetDevice(cur);
    if (e != hipSuccess || !p)
      return fail(SE_EHIP, "device address of the static scratch on device %d: %s", dev,
                  hipGetErrorString(e));
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return SE_OK;
}

static bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// Declared transform parts: known kinds, inside [0, K), disjoint, areas up to
// 64 x 64 (powers of two for Walsh-Hadamard); an area of T frames is
// transformed with its frames stacked, so T M <= 64.  A complex dictionary
// declares at most one part, a DFT part on a two-dimensional area; a real
// one declares none.
static se_status check_parts(int T, int M, int N, int K, int n_parts, const se_part* parts,
                             bool complex_dict) {
  if (n_parts < 0 || n_parts > 2) return fail(SE_EINVAL, "n_parts=%d must be 0, 1 or 2", n_parts);
  if (n_parts == 0) return SE_OK;
  for (int q = 0; q < n_parts; ++q)
    if ((parts[q].kind == SE_PART_DFT2) != complex_dict)
      return fail(SE_EINVAL, complex_dict ? "part %d: complex dictionaries take DFT parts only"
                                          : "part %d: a DFT part needs a complex dictionary",
                  q);
  if (complex_dict) {
    if (n_parts != 1) return fail(SE_EINVAL, "a complex dictionary declares at most one part");
    if (T != 1) return fail(SE_EINVAL, "DFT parts take two-dimensional areas");
  }
  if ((long long)T * M > 64 || N > 64)
    return fail(SE_EINVAL, "transform parts need T M, N <= 64 (got %dx%dx%d)", T, M, N);
  if (T > 1 && !is_pow2(M))
    return fail(SE_EINVAL, "transform parts of areas of several frames need a power-of-two M");
  const int P = T * M * N;
  for (int q = 0; q < n_parts; ++q) {
    const se_part& p = parts[q];
    if (p.kind != SE_PART_DCT2 && p.kind != SE_PART_WHT2 && p.kind != SE_PART_DFT2)
      return fail(SE_EINVAL, "part %d: unknown kind %d", q, p.kind);
    if (p.kind == SE_PART_WHT2 && (!is_pow2(T) || !is_pow2(M) || !is_pow2(N)))
      return fail(SE_EINVAL, "part %d: Walsh-Hadamard needs power-of-two T, M, N", q);
    if (p.first < 0 || (long long)p.first + P > K)
      return fail(SE_EINVAL, "part %d: atoms %d .. %d outside the dictionary", q, p.first,
                  p.first + P - 1);
  }
  if (n_parts == 2 && parts[0].first < parts[1].first + P && parts[1].first < parts[0].first + P)
    return fail(SE_EINVAL, "parts overlap");
  return SE_OK;
}

se_status check_basis_parts(const se_basis* b) {
  return check_parts(area_frames(b->T), b->M, b->N, b->K, b->n_parts, b->parts,
                     b->phi_im != nullptr);
}

static se_status check_tables(const se_tables* t) {
  if (!t) return fail(SE_EINVAL, "tables is NULL");
  if (t->M < 1 || t->N < 1 || t->K < 1 || t->T < 0)
    return fail(SE_EINVAL, "bad table shape T=%d M=%d N=%d K=%d", t->T, t->M, t->N, t->K);
  if ((long long)area_frames(t->T) * t->M * t->N > (1 << 24)) return fail(SE_EINVAL, "area too large");
  if (greedy_waves_for(t->K) == 0) return fail(SE_EINVAL, "K=%d exceeds %d", t->K, 32768);
  if (t->ldG < greedy_row_len(t->K) || (t->ldG & 3))
    return fail(SE_EINVAL, "ldG=%d must be >= se_table_ld(K)=%d and a multiple of 4", t->ldG,
                greedy_row_len(t->K));
  if (!t->G || !t->D || !t->Y || !t->sqrtw || !t->phi) return fail(SE_EINVAL, "a table pointer is NULL");
  if (reinterpret_cast<uintptr_t>(t->G) % 16) return fail(SE_EINVAL, "G must be 16-byte aligned");
  if (t->precision != SE_FP32 && t->precision != SE_BF16X3)
    return fail(SE_EINVAL, "unknown table precision %d", t->precision);
  if (t->precision == SE_BF16X3 && (!t->Yhi || !t->Ylo))
    return fail(SE_EINVAL, "BF16X3 tables need Yhi and Ylo");
  se_status st = check_parts(area_frames(t->T), t->M, t->N, t->K, t->n_parts, t->parts,
                             t->phi_im != nullptr);
  if (st) return st;
  if (t->n_parts > 0 && (!t->tx || reinterpret_cast<uintptr_t>(t->tx) % 16))
    return fail(SE_EINVAL, "tables with transform parts need a 16-byte aligned tx buffer");
  if (t->phi_im) {
    if (t->precision != SE_FP32) return fail(SE_EINVAL, "complex dictionaries take FP32 tables");
    if (!t->G_im || reinterpret_cast<uintptr_t>(t->G_im) % 16)
      return fail(SE_EINVAL, "complex tables need a 16-byte aligned G_im");
    if (!complex_loop_for(t->K)) return fail(SE_EINVAL, "no complex loop shape for K=%d", t->K);
    if (area_frames(t->T) > 1) return fail(SE_EINVAL, "complex dictionaries take two-dimensional areas");
  }
  if (t->n_classes != 0) {
    if (t->n_classes != 4 || !classes_possible(t) ||
        reinterpret_cast<uintptr_t>(t->Gc) % 16 || reinterpret_cast<uintptr_t>(t->cls) % 16)
      return fail(SE_EINVAL, "n_classes=%d does not describe class tables of these tables",
                  t->n_classes);
  }
  return SE_OK;
}

// Row length of R for the tables: real parts, and for a complex dictionary
// the imaginary parts after them.
static int r_row_len(const se_tables* t) {
  return (t->phi_im ? 2 : 1) * greedy_row_len(t->K);
}

static se_status check_r(const se_tables* t, const float* R, int ldR) {
  const int need = r_row_len(t), mult = t->phi_im ? 8 : 4;
  if (!R || ldR < need || ldR % mult || reinterpret_cast<uintptr_t>(R) % 16)
    return fail(SE_EINVAL, "R must be 16-byte aligned with ldR >= %d, a multiple of %d", need,
                mult);
  return SE_OK;
}

static inline int round8(int v) { return (v + 7) & ~7; }

// Partial products when the FP32 projection splits its contraction (few
// blocks): sized for rows of the minimum table row length.
// (partial products of the automatic split (mode 0), of the fixed split of
// SE_INVARIANT (mode 1), or whichever is larger (mode 2: the public sizes,
// which do not know the flags))
static size_t project_splitk_floats(const se_tables* t, int n_blk, int mode = 2) {
  const int P = area_samples(t);
  auto room = [&](int Mst) {
    const size_t a = mode == 1 ? 0 : gemm_splitk_floats(Mst, n_blk, P);
    const size_t b = mode == 0 ? 0 : gemm_invariant_floats(Mst, n_blk, P);
    return std::max(a, b);
  };
  if (t->n_parts == 0) return room(greedy_row_len(t->K));
  if (t->n_parts > 2) return 0;
  int lo[3], hi[3];
  const int nr = dense_ranges(t->K, P, t->n_parts, t->parts, lo, hi);
  size_t f = 0;
  for (int r = 0; r < nr; ++r) f = std::max(f, room(hi[r] - lo[r]));
  return f;
}

// Workspace of the projection stage: X as float32 (and the partial
// products), or as split bf16 pairs.
static size_t project_ws(const se_tables* t, int n_blk, int mode = 2) {
  Carver cv(nullptr);
  const int P = area_samples(t);
  if (t->precision == SE_BF16X3) {
    cv.take<uint16_t>((size_t)n_blk * round8(P));
    cv.take<uint16_t>((size_t)n_blk * round8(P));
  } else {
    cv.take<float>((size_t)n_blk * round4(P));
    cv.take<float>(project_splitk_floats(t, n_blk, mode));
  }
  return cv.off + 256;
}

// Atom ranges [lo, hi) not covered by transform parts.
int dense_ranges(int K, int P, int n_parts, const se_part* parts, int lo[3], int hi[3]) {
  int f[2] = {0, 0}, n = n_parts;
  for (int q = 0; q < n; ++q) f[q] = parts[q].first;
  if (n == 2 && f[1] < f[0]) std::swap(f[0], f[1]);
  int c = 0, r = 0;
  for (int q = 0; q < n; ++q) {
    if (f[q] > c) { lo[r] = c; hi[r] = f[q]; ++r; }
    c = f[q] + P;
  }
  if (c < K) { lo[r] = c; hi[r] = K; ++r; }
  return r;
}

// Checks every atom of the declared parts against phi on the device and
// waits for the verdict (flag: one device int32 of scratch).  With extra,
// the int32 after the flag (written by work the caller queued after
// clearing it) is read back in the same synchronisation.
static se_status verify_parts(const se_basis* b, int32_t* flag, hipStream_t s,
                              int32_t* extra = nullptr) {
  if (b->n_parts == 0) return SE_OK;
  se_status st;
  if (hipMemsetAsync(flag, 0, sizeof(int32_t), s) != hipSuccess)
    return fail(SE_EHIP, "flag clear failed");
  for (int q = 0; q < b->n_parts; ++q)
    if ((st = b->parts[q].kind == SE_PART_DFT2
                  ? check_dft_part(b->phi, b->phi_im, b->M, b->N, b->parts[q].first, flag, s)
                  : check_part(b->phi, area_frames(b->T), b->M, b->N, b->parts[q].kind,
                               b->parts[q].first, flag, s)))
      return st;
  int32_t got[2] = {0, 0};
  if (hipMemcpyAsync(got, flag, (extra ? 2 : 1) * sizeof(int32_t), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(SE_EHIP, "part verification: %s", hipGetErrorString(hipGetLastError()));
  if (extra) *extra = got[1];
  if (got[0]) return fail(SE_EINVAL, "a declared transform part does not match phi");
  return SE_OK;
}

// gather + projection GEMM in the tables' precision, over the dense atoms;
// the transform parts as separable transforms.  ws holds project_ws().
static se_status project_into(const se_tables* t, const uint8_t* images, int H, int W,
                              const se_block* dblk, int n_blk, float* R, int ldR, void* ws,
                              hipStream_t s, bool invariant = false) {
  se_status st;
  const int P = area_samples(t);
  int lo[3] = {0, 0, 0}, hi[3] = {t->K, 0, 0};
  int nr = 1;
  if (t->n_parts > 0) {
    // a complex DFT part writes its own columns only (R's two halves); the
    // padding is written below
    st = t->phi_im ? project_dft(t, images, H, W, dblk, n_blk, R, ldR, ldR / 2, s)
                   : project_tx(t, images, H, W, dblk, n_blk, R, ldR, s);
    if (st) return st;
    nr = dense_ranges(t->K, P, t->n_parts, t->parts, lo, hi);
    if (nr == 0 && !t->phi_im) return SE_OK;
  }
  if (t->phi_im && nr == 0) {
    launch_zero_range(R, n_blk, ldR, t->K, ldR / 2, s);
    launch_zero_range(R, n_blk, ldR, ldR / 2 + t->K, ldR, s);
    return check_launch("zero_range");
  }
  const bool pad = t->n_parts == 0;   // else the transform kernel wrote the padding
  Carver cv(ws);
  if (t->precision == SE_BF16X3) {
    const int ldX = round8(P);
    uint16_t* xh = cv.take<uint16_t>((size_t)n_blk * ldX);
    uint16_t* xl = cv.take<uint16_t>((size_t)n_blk * ldX);
    launch_gather_split(images, H, W, dblk, n_blk, area_frames(t->T), t->M, t->N, t->sqrtw, xh, xl,
                        ldX, s);
    if ((st = check_launch("gather_split"))) return st;
    for (int r = 0; r < nr; ++r) {
      const size_t off = (size_t)lo[r] * P;
      if ((st = gemm_project_bf16x3(t->Yhi + off, t->Ylo + off, P, hi[r] - lo[r], xh, xl, ldX,
                                    n_blk, P, R + lo[r], ldR, s, pad)))
        return st;
    }
    return SE_OK;
  }
  const int ldX = round4(P);
  float* X = cv.take<float>((size_t)n_blk * ldX);
  // invariant: the contraction split into slices fixed by the number of
  // samples, not by the number of blocks (the automatic split depends on the
  // batch size, which would change the rounding)
  const size_t split_floats = project_splitk_floats(t, n_blk, invariant ? 1 : 0);
  float* split = cv.take<float>(split_floats);
  const int split_rule = invariant ? kSplitShape : -1;
  launch_gather(images, H, W, dblk, n_blk, area_frames(t->T), t->M, t->N, t->sqrtw, X, ldX, s);
  if ((st = check_launch("gather"))) return st;
  if (t->phi_im) {
    // complex dictionary: real and imaginary parts of eq. 12 from the two
    // halves of Y, into the two halves of each row of R (the atoms outside
    // a DFT part)
    const int K = t->K, half = ldR / 2;
    for (int part = 0; part < 2; ++part)
      for (int r = 0; r < nr; ++r)
        if ((st = gemm_project_f32(t->Y + ((size_t)part * K + lo[r]) * P, P, hi[r] - lo[r], X,
                                   ldX, n_blk, P, R + part * half + lo[r], ldR, 0, s, false, split,
                                   split_floats, split_rule)))
          return st;
    launch_zero_range(R, n_blk, ldR, K, half, s);
    launch_zero_range(R, n_blk, ldR, half + K, ldR, s);
    return check_launch("zero_range");
  }
  const int tile = tune_lookup(t->K, P, n_blk).proj_tile;
  for (int r = 0; r < nr; ++r)
    if ((st = gemm_project_f32(t->Y + (size_t)lo[r] * P, P, hi[r] - lo[r], X, ldX, n_blk, P,
                               R + lo[r], ldR, tile, s, pad, split, split_floats, split_rule)))
      return st;
  return SE_OK;
}

// Each block writes its loss into the images in place, so no pixel may lie
// in two losses.  The losses (clipped to the frames, which is all a block
// writes) are bucketed by the 32 x 32 cells of each frame they touch, and
// only losses that share a cell are compared: linear in the number of blocks.
// The buckets live in an open-addressing table of the calling thread, at
// most half full and reused across calls (a generation stamp marks the live
// slots, so nothing is cleared per call).
static se_status check_loss_overlap(const se_block* blocks, int n_blk, int H, int W) {
  struct Box {
    int f0, f1, y0, y1, x0, x1;   // inclusive; y1 < y0 when wholly outside
  };
  struct Slot {
    uint64_t key;
    uint32_t gen;
    int head;                     // newest entry of the cell
  };
  struct Entry {
    int box, next;
  };
  thread_local std::vector<Slot> tl_table;
  thread_local std::vector<Box> tl_box;
  thread_local std::vector<Entry> tl_entries;
  thread_local uint32_t tl_gen = 0;
  if (n_blk < 2) return SE_OK;
  // one thread-local lookup each (every access to a thread_local of a
  // shared library is a call)
  std::vector<Slot>& table = tl_table;
  std::vector<Box>& box = tl_box;
  std::vector<Entry>& entries = tl_entries;
  uint32_t& gen_ref = tl_gen;
  box.resize((size_t)n_blk);
  size_t n_cells = 0;
  for (int i = 0; i < n_blk; ++i) {
    const se_block& b = blocks[i];
    const int ld = b.ld < 1 ? 1 : b.ld;
    Box& q = box[(size_t)i];
    q = Box{b.img + b.lt, b.img + b.lt + ld - 1, std::max(b.y0 + b.ly, 0),
            std::min(b.y0 + b.ly + b.lh, H) - 1, std::max(b.x0 + b.lx, 0),
            std::min(b.x0 + b.lx + b.lw, W) - 1};
    if (q.y1 >= q.y0 && q.x1 >= q.x0)
      n_cells += (size_t)ld * ((q.y1 >> 5) - (q.y0 >> 5) + 1) * ((q.x1 >> 5) - (q.x0 >> 5) + 1);
  }
  size_t cap = 1024;
  while (cap < 2 * n_cells) cap <<= 1;
  if (table.size() < cap || ++gen_ref == 0) {
    table.assign(std::max(cap, table.size()), Slot{0, 0, -1});
    gen_ref = 1;
  }
  const uint32_t gen = gen_ref;
  const size_t mask = table.size() - 1;
  int shift = 64;                 // Fibonacci hashing: the product's top bits
  for (size_t c = table.size(); c > 1; c >>= 1) --shift;
  entries.clear();
  for (int i = 0; i < n_blk; ++i) {
    const Box& q = box[(size_t)i];
    if (q.y1 < q.y0 || q.x1 < q.x0) continue;
    for (int f = q.f0; f <= q.f1; ++f)
      for (int cy = q.y0 >> 5; cy <= q.y1 >> 5; ++cy)
        for (int cx = q.x0 >> 5; cx <= q.x1 >> 5; ++cx) {
          const uint64_t key = ((uint64_t)(uint32_t)f << 40) | ((uint64_t)(uint32_t)cy << 20) |
                               (uint64_t)(uint32_t)cx;
          size_t h = (size_t)((key * 0x9E3779B97F4A7C15ull) >> shift);
          while (table[h].gen == gen && table[h].key != key) h = (h + 1) & mask;
          Slot& sl = table[h];
          if (sl.gen != gen) sl = Slot{key, gen, -1};
          for (int e = sl.head; e >= 0; e = entries[(size_t)e].next) {
            const int j = entries[(size_t)e].box;
            const Box& o = box[(size_t)j];
            if (o.f0 <= q.f1 && q.f0 <= o.f1 && o.y0 <= q.y1 && q.y0 <= o.y1 && o.x0 <= q.x1 &&
                q.x0 <= o.x1)
              return fail(SE_EINVAL, "blocks %d and %d: their losses overlap", j, i);
          }
          entries.push_back(Entry{i, sl.head});
          sl.head = (int)entries.size() - 1;
        }
  }
  return SE_OK;
}

static se_status check_blocks(const se_tables* t, int n_img, int H, int W, const se_block* blocks,
                              int n_blk, int g_loss_ld, const float* g_loss) {
  if (n_blk < 0) return fail(SE_EINVAL, "n_blk < 0");
  if (n_blk > 0 && !blocks) return fail(SE_EINVAL, "blocks is NULL");
  if (n_img < 1 || H < 1 || W < 1) return fail(SE_EINVAL, "bad image batch %d x %d x %d", n_img, H, W);
  const int T = 64 * greedy_waves_for(t->K), F = area_frames(t->T);
  for (int i = 0; i < n_blk; ++i) {
    const se_block& b = blocks[i];
    if (b.img < 0 || (long long)b.img + F > n_img)
      return fail(SE_EINVAL, "block %d: frames %d .. %d out of range", i, b.img, b.img + F - 1);
    if (b.lh < 1 || b.lw < 1 || b.ly < 0 || b.lx < 0 || b.ly + b.lh > t->M || b.lx + b.lw > t->N)
      return fail(SE_EINVAL, "block %d: loss rectangle not inside the %dx%d area", i, t->M, t->N);
    const int ld = b.ld < 1 ? 1 : b.ld;
    if (b.lt < 0 || b.lt + ld > F)
      return fail(SE_EINVAL, "block %d: loss frames %d .. %d not inside the %d frames of the area",
                  i, b.lt, b.lt + ld - 1, F);
    const long long n = (long long)ld * b.lh * b.lw;
    if (n > 4 * T) return fail(SE_EINVAL, "block %d: loss of %lld pixels exceeds %d", i, n, 4 * T);
    if (g_loss && n > g_loss_ld)
      return fail(SE_EINVAL, "block %d: g_loss_ld=%d < loss size %lld", i, g_loss_ld, n);
  }
  return check_loss_overlap(blocks, n_blk, H, W);
}

}  // namespace sefase

using namespace sefase;

extern "C" {

const char* se_last_error(void) { return g_err; }
int32_t se_version(void) { return 100; }
int32_t se_table_ld(int32_t K) { return K >= 1 && greedy_waves_for(K) ? greedy_row_len(K) : 0; }
size_t se_tables_tx_bytes(int32_t M, int32_t N, int32_t n_parts) {
  // room for two transforms: a DFT part is stored as its real and its
  // imaginary transform
  return n_parts == 1 || n_parts == 2 ? tx_const_bytes(M, N, 2) : 0;
}

// ---------------------------------------------------------------------------
size_t se_area_weights_ws_bytes(int32_t n_blk) {
  return align_up((size_t)(n_blk > 0 ? n_blk : 0) * sizeof(DevBlock), 256) + 256;
}

se_status se_volume_weights(int32_t T, int32_t M, int32_t N, float rho_hat, const uint8_t* lost,
                            int32_t n_img, int32_t H, int32_t W, const se_block* blocks,
                            int32_t n_blk, float* w, void* ws, size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  if (T < 1 || M < 1 || N < 1) return fail(SE_EINVAL, "bad area %dx%dx%d", T, M, N);
  if ((long long)T * M * N > (1 << 24)) return fail(SE_EINVAL, "area too large");
  if (!(rho_hat > 0.0f && rho_hat <= 1.0f)) return fail(SE_EINVAL, "rho_hat must lie in (0, 1]");
  if (!lost || !w || (n_blk > 0 && !blocks)) return fail(SE_EINVAL, "NULL pointer");
  if (n_img < 1 || H < 1 || W < 1) return fail(SE_EINVAL, "bad image batch");
  if (n_blk < 0) return fail(SE_EINVAL, "n_blk < 0");
  for (int i = 0; i < n_blk; ++i)
    if (blocks[i].img < 0 || (long long)blocks[i].img + T > n_img)
      return fail(SE_EINVAL, "block %d: frames %d .. %d out of range", i, blocks[i].img,
                  blocks[i].img + T - 1);
  if (n_blk == 0) return SE_OK;
  if (!ws || ws_bytes < se_area_weights_ws_bytes(n_blk)) return fail(SE_ENOMEM, "workspace too small");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Carver cv(ws);
  DevBlock* dblk = cv.take<DevBlock>((size_t)n_blk);
  se_status st = upload_blocks(blocks, n_blk, dblk, s);
  if (st) return st;
  launch_area_weights(T, M, N, rho_hat, lost, H, W, dblk, n_blk, w, s);
  return check_launch("area_weights");
}

se_status se_area_weights(int32_t M, int32_t N, float rho_hat, const uint8_t* lost, int32_t n_img,
                          int32_t H, int32_t W, const se_block* blocks, int32_t n_blk, float* w,
                          void* ws, size_t ws_bytes, void* stream) {
  return se_volume_weights(1, M, N, rho_hat, lost, n_img, H, W, blocks, n_blk, w, ws, ws_bytes,
                           stream);
}

// ---------------------------------------------------------------------------
size_t se_weighted_gram_ws_bytes(const se_basis* b, se_precision prec) {
  (void)prec;
  if (!b || b->K < 1 || b->M < 1 || b->N < 1) return 0;
  Carver cv(nullptr);
  const size_t K = (size_t)b->K;
  cv.take<float>(K);
  cv.take<double>(K);
  cv.take<int32_t>(2);
  if (b->phi_im) cv.take<float>(2 * K * (size_t)round4(2 * b->K));   // the stacked product
  return cv.off + 256;
}

se_status se_weighted_gram(const se_basis* b, const float* w, se_precision prec, uint32_t flags,
                           se_tables* t, void* ws, size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  if (!b || !w || !t) return fail(SE_EINVAL, "NULL argument");
  if (!b->phi) return fail(SE_EINVAL, "basis phi is NULL");
  if (b->M < 1 || b->N < 1 || b->K < 1) return fail(SE_EINVAL, "bad basis shape");
  if (prec != SE_FP32 && prec != SE_BF16X3) return fail(SE_EINVAL, "unknown precision %d", (int)prec);
  if (flags > SE_DIAG_FP32) return fail(SE_EINVAL, "unknown flags 0x%x", flags);
  if (reinterpret_cast<uintptr_t>(t->Gq) % 16) return fail(SE_EINVAL, "Gq must be 16-byte aligned");
  if (reinterpret_cast<uintptr_t>(t->Gq_rows) % 16)
    return fail(SE_EINVAL, "Gq_rows must be 16-byte aligned");
  t->M = b->M;
  t->N = b->N;
  t->K = b->K;
  t->phi = b->phi;
  t->precision = (int32_t)prec;
  t->n_parts = b->n_parts;
  for (int q = 0; q < 2; ++q) t->parts[q] = q < b->n_parts ? b->parts[q] : se_part{0, 0};
  t->phi_im = b->phi_im;
  t->T = area_frames(b->T);
  t->n_classes = 0;
  se_status st = check_tables(t);
  if (st) return st;
  if (!ws || ws_bytes < se_weighted_gram_ws_bytes(b, prec)) return fail(SE_ENOMEM, "workspace too small");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int K = b->K, P = area_samples(t);
  Carver cv(ws);
  float* diag32 = cv.take<float>((size_t)K);
  double* diag64 = cv.take<double>((size_t)K);
  int32_t* flag = cv.take<int32_t>(2);
  // the projections of declared parts are computed from their definition,
  // so the declaration must match the atoms actually given; the weight
  // pattern's mirror symmetry (for class tables) is read back in the same
  // synchronisation
  const bool want_classes = classes_possible(t);
  int32_t asym = 1;
  if (want_classes) {
    if (hipMemsetAsync(flag + 1, 0, sizeof(int32_t), s) != hipSuccess)
      return fail(SE_EHIP, "flag clear failed");
    launch_sym_check(w, area_frames(b->T), b->M, b->N, flag + 1, s);
    if ((st = check_launch("sym_check"))) return st;
  }
  if ((st = verify_parts(b, flag, s, want_classes ? &asym : nullptr))) {
    t->n_parts = 0;
    return st;
  }
  launch_diag(b->phi, b->phi_im, w, K, P, diag32, diag64, s);
  if ((st = check_launch("diag"))) return st;
  launch_finalize_d(diag32, diag64, w, K, P, (int)flags, prec == SE_BF16X3 ? 1 : 0, t->D, t->sqrtw,
                    t->info, s);
  if ((st = check_launch("finalize_d"))) return st;
  if (b->phi_im) {
    // complex dictionary: Y = D sqrt(w) conj(phi) as stacked real and
    // imaginary rows; G = Y Y^H from their symmetric product (Algorithm 2's
    // Hermitian mirror is exact: Re G symmetric, Im G antisymmetric)
    launch_scale_y(b->phi, t->D, t->sqrtw, K, P, t->Y, s);
    launch_scale_y(b->phi_im, t->D, t->sqrtw, K, P, t->Y + (size_t)K * P, s, true);
    if ((st = check_launch("scale_y"))) return st;
    // a DFT part's projections are transforms (its operands from D and w);
    // the table itself stays the product of all atoms
    if (t->n_parts > 0 && (st = build_tx(t, s))) return st;
    launch_zero_cols(t->G, K, K, t->ldG, s);
    launch_zero_cols(t->G_im, K, K, t->ldG, s);
    if ((st = check_launch("zero_cols"))) return st;
    const int ldS = round4(2 * K);
    float* S = cv.take<float>((size_t)2 * K * ldS);
    if ((st = gemm_syrk_f32(t->Y, P, 2 * K, P, S, ldS, s))) return st;
    launch_combine_c(S, ldS, K, t->G, t->G_im, t->ldG, s);
    return check_launch("combine_c");
  }
  launch_scale_y(b->phi, t->D, t->sqrtw, K, P, t->Y, s);
  if ((st = check_launch("scale_y"))) return st;
  if (t->n_parts > 0 && (st = build_tx(t, s))) return st;
  launch_zero_cols(t->G, K, K, t->ldG, s);
  if ((st = check_launch("zero_cols"))) return st;
  if (prec == SE_BF16X3) {
    launch_split_bf16(t->Y, (size_t)K * P, t->Yhi, t->Ylo, s);
    if ((st = check_launch("split_bf16"))) return st;
  }
  // With transform parts and at most one dense range (starting on a 4-float
  // boundary), every row over the part columns is a transform of the
  // weighted atom (Section VI), the dense x dense block is the product of the
  // dense atoms, and a mirror pass fills the parts' rows over the dense
  // columns; otherwise the whole table is one symmetric product.
  int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  const int nr = t->n_parts > 0 ? dense_ranges(K, P, t->n_parts, t->parts, lo, hi) : 3;
  if (nr <= 1 && (lo[0] & 3) == 0) {
    if ((st = gram_tx(t, s))) return st;
    if (nr == 1) {
      const int kd = hi[0] - lo[0];
      float* Gd = t->G + (size_t)lo[0] * t->ldG + lo[0];
      st = prec == SE_FP32
               ? gemm_syrk_f32(t->Y + (size_t)lo[0] * P, P, kd, P, Gd, t->ldG, s)
               : gemm_syrk_bf16x3(t->Yhi + (size_t)lo[0] * P, t->Ylo + (size_t)lo[0] * P, P, kd, P,
                                  Gd, t->ldG, s);
      if (st) return st;
    }
    if ((st = gram_mirror(t, s))) return st;
    if (want_classes && asym == 0) {
      if ((st = build_classes(t, s))) return st;
      if (t->Gq && (st = quantise_classes(t, s))) return st;
      t->n_classes = 4;
    }
  } else {
    st = prec == SE_FP32 ? gemm_syrk_f32(t->Y, P, K, P, t->G, t->ldG, s)
                         : gemm_syrk_bf16x3(t->Yhi, t->Ylo, P, K, P, t->G, t->ldG, s);
    if (st) return st;
  }
  // fixed-point words of every whole row (real tables)
  if (t->Gq_rows && (st = quantise_rows(t, s))) return st;
  return SE_OK;
}

// ---------------------------------------------------------------------------
se_status se_blocks_upload(const se_tables* t, int32_t n_img, int32_t H, int32_t W,
                           const se_block* blocks, int32_t n_blk, se_block* dev_blocks,
                           int32_t* max_loss, void* stream) {
  g_err[0] = 0;
  se_status st = check_tables(t);
  if (st) return st;
  if ((st = check_blocks(t, n_img, H, W, blocks, n_blk, 0, nullptr))) return st;
  int mx = 0;
  for (int i = 0; i < n_blk; ++i)
    mx = std::max(mx, (blocks[i].ld < 1 ? 1 : blocks[i].ld) * blocks[i].lh * blocks[i].lw);
  if (max_loss) *max_loss = mx;
  if (n_blk == 0) return SE_OK;
  if (!dev_blocks) return fail(SE_EINVAL, "dev_blocks is NULL");
  const AreaShape sh{H, W, area_frames(t->T), t->M, t->N};
  int n_deg = 0;
  if ((st = upload_blocks(blocks, n_blk, dev_blocks, static_cast<hipStream_t>(stream), &sh,
                          &n_deg)))
    return st;
  return degenerate_status(n_deg);
}

size_t se_project_ws_bytes(const se_tables* t, int32_t n_blk) {
  if (!t || t->K < 1 || t->M < 1 || t->N < 1 || n_blk < 0) return 0;
  return project_ws(t, n_blk);
}

static se_status check_common(const se_tables* t, int n_img, int H, int W, int n_blk,
                              const void* images, const void* dev_blocks) {
  se_status st = check_tables(t);
  if (st) return st;
  if (n_img < 1 || H < 1 || W < 1) return fail(SE_EINVAL, "bad image batch %d x %d x %d", n_img, H, W);
  if (n_blk < 0) return fail(SE_EINVAL, "n_blk < 0");
  if (n_blk > 0 && (!images || !dev_blocks)) return fail(SE_EINVAL, "NULL pointer");
  return SE_OK;
}

se_status se_project(const se_tables* t, const uint8_t* images, int32_t n_img, int32_t H, int32_t W,
                     const se_block* dev_blocks, int32_t n_blk, float* R, int32_t ldR, void* ws,
                     size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  se_status st = check_common(t, n_img, H, W, n_blk, images, dev_blocks);
  if (st) return st;
  if (n_blk == 0) return SE_OK;
  if ((st = check_r(t, R, ldR))) return st;
  if (!ws || ws_bytes < se_project_ws_bytes(t, n_blk)) return fail(SE_ENOMEM, "workspace too small");
  return project_into(t, images, H, W, dev_blocks, n_blk, R, ldR, ws,
                      static_cast<hipStream_t>(stream));
}

static GreedyArgs greedy_args(const se_tables* t, const float* R, int ldR, uint8_t* images, int H,
                              int W, const se_block* dev_blocks, int n_blk, se_params prm,
                              int32_t* sel, float* coef, float* g_loss, int g_loss_ld) {
  GreedyArgs ga;
  ga.R0 = R;
  ga.ldR = ldR;
  ga.G = t->G;
  ga.ldG = t->ldG;
  ga.D = t->D;
  ga.phi = t->phi;
  ga.K = t->K;
  ga.M = t->M;
  ga.N = t->N;
  ga.P = area_samples(t);
  ga.blk = dev_blocks;
  ga.n_blk = n_blk;
  ga.blk0 = -1;   // batched: block = workgroup index
  ga.images = images;
  ga.H = H;
  ga.W = W;
  ga.gamma = prm.gamma;
  ga.iters = prm.iters;
  ga.sel = sel;
  ga.coef = coef;
  ga.g_loss = g_loss;
  ga.g_loss_ld = g_loss ? g_loss_ld : 0;
  ga.Gc = t->n_classes == 4 ? t->Gc : nullptr;
  ga.cls = t->n_classes == 4 ? reinterpret_cast<const int2*>(t->cls) : nullptr;
  ga.Gq = (prm.flags & SE_ROWS_Q14) && t->n_classes == 4 ? t->Gq : nullptr;
  ga.Gqr = (prm.flags & SE_ROWS_Q14) && !t->phi_im ? t->Gq_rows : nullptr;
  ga.cl = t->n_classes == 4 ? class_layout(t) : ClassLayout{};
  ga.n_degenerate = nullptr;
  return ga;
}

// the loop for the tables' kind: real (the tuned or default shape) or complex
static se_status launch_loop(const se_tables* t, const GreedyArgs& ga, int n_blk, hipStream_t s,
                             const TuneChoice& tc) {
  if (t->phi_im) return launch_greedy_c(ga, t->G_im, t->phi_im, n_blk, s);
  return launch_greedy(ga, n_blk, s, tc.loop_waves, tc.loop_vpl);
}

static se_status check_params(se_params prm, const float* g_loss, int g_loss_ld) {
  if (!(prm.gamma > 0.0f && prm.gamma <= 1.0f)) return fail(SE_EINVAL, "gamma must lie in (0, 1]");
  if (prm.iters < 0) return fail(SE_EINVAL, "iters < 0");
  if (prm.flags & ~(SE_ROWS_Q14 | SE_ROWS_BF16X3 | SE_INVARIANT))
    return fail(SE_EINVAL, "unknown flags 0x%x", prm.flags);
  if (g_loss && g_loss_ld < 1) return fail(SE_EINVAL, "g_loss_ld < 1");
  return SE_OK;
}

// The flags of the table routes: SE_ROWS_Q14 reads the class words Gq on the
// one-launch route (one_launch: the call takes it for these tables) and the
// whole-row words Gq_rows on the loop over whole rows; SE_ROWS_BF16X3
// belongs to rows on demand.
static se_status check_route_flags(const se_tables* t, se_params prm, bool one_launch) {
  if (prm.flags & SE_ROWS_BF16X3)
    return fail(SE_EINVAL, "SE_ROWS_BF16X3 is an option of rows on demand");
  if (!(prm.flags & SE_ROWS_Q14)) return SE_OK;
  if (one_launch) {
    if (t->n_classes != 4)
      return fail(SE_EINVAL, "SE_ROWS_Q14 on the one-launch route needs class tables");
    if (!t->Gq || reinterpret_cast<uintptr_t>(t->Gq) % 16)
      return fail(SE_EINVAL, "SE_ROWS_Q14 needs 16-byte aligned fixed-point rows Gq");
    return SE_OK;
  }
  if (t->phi_im) return fail(SE_EINVAL, "SE_ROWS_Q14 takes real tables");
  if (!t->Gq_rows || reinterpret_cast<uintptr_t>(t->Gq_rows) % 16)
    return fail(SE_EINVAL,
                "SE_ROWS_Q14 on the loop over whole rows needs 16-byte aligned words Gq_rows");
  return SE_OK;
}

se_status se_iterate(const se_tables* t, const float* R, int32_t ldR, uint8_t* images, int32_t n_img,
                     int32_t H, int32_t W, const se_block* dev_blocks, int32_t n_blk, se_params prm,
                     int32_t* sel, float* coef, float* g_loss, int32_t g_loss_ld, void* stream) {
  g_err[0] = 0;
  se_status st = check_common(t, n_img, H, W, n_blk, images, dev_blocks);
  if (st) return st;
  if ((st = check_params(prm, g_loss, g_loss_ld))) return st;
  if ((st = check_route_flags(t, prm, false))) return st;
  if (n_blk == 0) return SE_OK;
  if ((st = check_r(t, R, ldR))) return st;
  GreedyArgs ga = greedy_args(t, R, ldR, images, H, W, dev_blocks, n_blk, prm, sel, coef, g_loss,
                              g_loss_ld);
  const TuneChoice tc = tune_lookup(t->K, area_samples(t), n_blk);
  return launch_loop(t, ga, n_blk, static_cast<hipStream_t>(stream), tc);
}

size_t se_extrapolate_device_ws_bytes(const se_tables* t, int32_t n_blk) {
  if (!t || t->K < 1 || t->M < 1 || t->N < 1 || n_blk < 0) return 0;
  if (conceal_tx_supported(t)) return 0;
  Carver cv(nullptr);
  cv.take<float>((size_t)n_blk * r_row_len(t));
  cv.take<char>(project_ws(t, n_blk));
  return cv.off + 256;
}

se_status se_extrapolate_device(const se_tables* t, uint8_t* images, int32_t n_img, int32_t H,
                                int32_t W, const se_block* dev_blocks, int32_t n_blk,
                                se_params prm, int32_t* sel, float* coef, float* g_loss,
                                int32_t g_loss_ld, void* ws, size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  se_status st = check_common(t, n_img, H, W, n_blk, images, dev_blocks);
  if (st) return st;
  if ((st = check_params(prm, g_loss, g_loss_ld))) return st;
  if ((st = check_route_flags(t, prm, conceal_tx_supported(t)))) return st;
  if (n_blk == 0) return SE_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int ldR = r_row_len(t);
  const TuneChoice tc = tune_lookup(t->K, area_samples(t), n_blk);
  if (conceal_tx_supported(t)) {
    const GreedyArgs ga = greedy_args(t, nullptr, ldR, images, H, W, dev_blocks, n_blk, prm, sel,
                                      coef, g_loss, g_loss_ld);
    return conceal_tx(t, ga, images, H, W, n_blk, s, tc.loop_waves, tc.loop_vpl);
  }
  const size_t need = se_extrapolate_device_ws_bytes(t, n_blk);
  if (!ws || ws_bytes < need) return fail(SE_ENOMEM, "workspace too small: need %zu bytes", need);
  Carver cv(ws);
  float* R = cv.take<float>((size_t)n_blk * ldR);
  char* pws = cv.take<char>(project_ws(t, n_blk));
  if ((st = project_into(t, images, H, W, dev_blocks, n_blk, R, ldR, pws, s,
                        (prm.flags & SE_INVARIANT) != 0)))
    return st;
  const GreedyArgs ga = greedy_args(t, R, ldR, images, H, W, dev_blocks, n_blk, prm, sel, coef,
                                    g_loss, g_loss_ld);
  return launch_loop(t, ga, n_blk, s, tc);
}

size_t se_extrapolate_batch_ws_bytes(const se_tables* t, int32_t n_blk) {
  if (!t || t->K < 1 || t->M < 1 || t->N < 1 || n_blk < 0) return 0;
  Carver cv(nullptr);
  cv.take<se_block>((size_t)n_blk);
  cv.take<float>((size_t)n_blk * r_row_len(t));
  cv.take<char>(project_ws(t, n_blk > 0 ? n_blk : 0));
  return cv.off + 256;
}

// Workspace one batched call actually uses on its route: the descriptors,
// and R with the projection workspace unless the projections stay in the
// loop's workgroups.
// (the exact need of one call: the split room of its own flag)
static size_t batch_route_ws(const se_tables* t, int n_blk, bool invariant) {
  Carver cv(nullptr);
  cv.take<se_block>((size_t)n_blk);
  if (!conceal_tx_supported(t)) {
    cv.take<float>((size_t)n_blk * r_row_len(t));
    cv.take<char>(project_ws(t, n_blk, invariant ? 1 : 0));
  }
  return cv.off;
}

static se_status extrapolate_uploaded(bool plain, const se_tables* t, uint8_t* images, int H,
                                      int W, se_block* dblk, float* R, char* pws, int n_blk,
                                      se_params prm, int32_t* sel, float* coef, float* g_loss,
                                      int32_t g_loss_ld, hipStream_t s, bool invariant);

// The batched and per-block calls.  use_static: the workspace is the static
// scratch of this device (ws ignored), sized for the route taken, and the
// descriptors are uploaded without a host staging buffer.
static se_status extrapolate(bool plain, const se_tables* t, uint8_t* images, int32_t n_img,
                             int32_t H, int32_t W, const se_block* blocks, int32_t n_blk,
                             se_params prm, int32_t* sel, float* coef, float* g_loss,
                             int32_t g_loss_ld, void* ws, size_t ws_bytes, void* stream,
                             bool use_static = false) {
  g_err[0] = 0;
  se_status st = check_tables(t);
  if (st) return st;
  if (!images) return fail(SE_EINVAL, "images is NULL");
  if ((st = check_params(prm, g_loss, g_loss_ld))) return st;
  if ((st = check_route_flags(t, prm, !plain && conceal_tx_supported(t)))) return st;
  if ((st = check_blocks(t, n_img, H, W, blocks, n_blk, g_loss_ld, g_loss))) return st;
  if (plain && t->phi_im) return fail(SE_EINVAL, "the per-block form takes real dictionaries");
  if (n_blk == 0) return SE_OK;
  const AreaShape sh{H, W, area_frames(t->T), t->M, t->N};
  const int n_deg = count_without_support(blocks, n_blk, sh);
  // nothing to compute and nothing to report on the device
  if (n_deg == n_blk && !sel && !coef && !g_loss) return degenerate_status(n_deg);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (use_static) {
    const size_t need = batch_route_ws(t, n_blk, (prm.flags & SE_INVARIANT) != 0);
    if (need > SE_STATIC_SCRATCH_BYTES)
      return fail(SE_ENOMEM, "the batch needs %zu bytes of scratch; the static scratch holds %zu",
                  need, (size_t)SE_STATIC_SCRATCH_BYTES);
    if ((st = static_scratch(s, &ws))) return st;
    ws_bytes = SE_STATIC_SCRATCH_BYTES;
  } else {
    const size_t need = se_extrapolate_batch_ws_bytes(t, n_blk);
    if (!ws || ws_bytes < need) return fail(SE_ENOMEM, "workspace too small: need %zu bytes", need);
  }
  const int ldR = r_row_len(t);
  Carver cv(ws);
  se_block* dblk = cv.take<se_block>((size_t)n_blk);
  float* R = cv.take<float>((size_t)n_blk * ldR);
  char* pws = cv.take<char>(project_ws(t, n_blk));
  if ((st = use_static ? upload_blocks_raw(blocks, n_blk, dblk, s, sh)
                       : upload_blocks(blocks, n_blk, dblk, s, &sh)))
    return st;
  if ((st = extrapolate_uploaded(plain, t, images, H, W, dblk, R, pws, n_blk, prm, sel, coef,
                                 g_loss, g_loss_ld, s, (prm.flags & SE_INVARIANT) != 0)))
    return st;
  return degenerate_status(n_deg);
}

// The launches of extrapolate() once the descriptors are on the device.
static se_status extrapolate_uploaded(bool plain, const se_tables* t, uint8_t* images, int H,
                                      int W, se_block* dblk, float* R, char* pws, int n_blk,
                                      se_params prm, int32_t* sel, float* coef, float* g_loss,
                                      int32_t g_loss_ld, hipStream_t s, bool invariant) {
  se_status st;
  const int P = area_samples(t), ldR = r_row_len(t);
  GreedyArgs ga = greedy_args(t, R, ldR, images, H, W, dblk, n_blk, prm, sel, coef, g_loss,
                              g_loss_ld);
  if (!plain) {
    const TuneChoice tc = tune_lookup(t->K, P, n_blk);
    if (conceal_tx_supported(t))   // projections inside the loop's workgroups
      return conceal_tx(t, ga, images, H, W, n_blk, s, tc.loop_waves, tc.loop_vpl);
    if ((st = project_into(t, images, H, W, dblk, n_blk, R, ldR, pws, s, invariant))) return st;
    return launch_loop(t, ga, n_blk, s, tc);
  }
  // one block at a time: gather, matrix-vector product (FP32), single-workgroup loop
  float* X = reinterpret_cast<float*>(pws);
  for (int i = 0; i < n_blk; ++i) {
    launch_gather(images, H, W, dblk + i, 1, area_frames(t->T), t->M, t->N, t->sqrtw, X, round4(P),
                  s);
    if ((st = check_launch("gather"))) return st;
    launch_gemv(t->Y, t->K, P, X, R, s);
    if ((st = check_launch("gemv"))) return st;
    ga.blk0 = i;
    if ((st = launch_greedy(ga, 1, s, 0, 0))) return st;
  }
  return SE_OK;
}

// ---------------------------------------------------------------------------
static inline int round1024(int v) { return (v + 1023) & ~1023; }

// workspace for the split products of the on-demand path: the per-block
// diagonal and projections (every atom, padded rows) and the per-iteration
// rows (the dense ranges when transform parts are declared); with `tuned`,
// room for any split the tuner may choose (up to 8 slices)
static size_t ondemand_splitk_floats(const se_basis* b, int n_blk, bool tuned = false) {
  const int P = b->M * b->N, ld = round1024(b->K);
  size_t f = gemm_splitk_floats(ld, n_blk, P);
  int lo[3] = {0, 0, 0}, hi[3] = {b->K, 0, 0};
  const int nr = b->n_parts > 0 && b->n_parts <= 2
                     ? dense_ranges(b->K, P, b->n_parts, b->parts, lo, hi)
                     : 1;
  f = std::max(f, gemm_invariant_floats(ld, n_blk, P));   // SE_INVARIANT's fixed split
  for (int r = 0; r < nr; ++r) {
    f = std::max(f, gemm_rows_splitk_floats(hi[r] - lo[r], n_blk, P, -1));
    f = std::max(f, gemm_rows_splitk_floats(hi[r] - lo[r], n_blk, P, kSplitShape));
    if (tuned) f = std::max(f, gemm_rows_splitk_floats(hi[r] - lo[r], n_blk, P, 8));
  }
  return f;
}

// The basis checks of rows on demand.
static se_status check_od_basis(const se_basis* b) {
  if (b && b->phi_im) return fail(SE_EINVAL, "rows on demand take real dictionaries");
  if (b && b->T > 1) return fail(SE_EINVAL, "rows on demand take two-dimensional areas");
  if (!b || !b->phi) return fail(SE_EINVAL, "NULL argument");
  if (b->M < 1 || b->N < 1 || b->K < 1) return fail(SE_EINVAL, "bad basis shape");
  if (b->K > 32768) return fail(SE_EINVAL, "K=%d exceeds 32768", b->K);
  if ((long long)b->M * b->N > (1 << 24)) return fail(SE_EINVAL, "area too large");
  return check_basis_parts(b);
}

// Workspace of a batch on demand, carved in one order for the size query
// (base NULL) and the call.  own_dict: the dictionary's own pieces (phi
// squared, transform operands, split copy, verification flag) live in the
// workspace too (se_extrapolate_ondemand); a prepared dictionary holds them.
struct OdCarve {
  se_block* dblk = nullptr;
  int32_t* dorig = nullptr;
  int32_t* flag = nullptr;
  float* tx = nullptr;
  uint16_t* phi_split = nullptr;
};
static void carve_ondemand(Carver& cv, const se_basis* b, int n_blk, int max_loss, int slots,
                           bool own_dict, bool bf16, bool tuned, OnDemandPlan& pl, OdCarve& oc) {
  const size_t K = (size_t)b->K, P = (size_t)b->M * b->N, n = (size_t)n_blk;
  const size_t ld = (size_t)round1024(b->K), ldV = (size_t)round4((int)P);
  const size_t ml = (size_t)(max_loss > 0 ? max_loss : 1);
  oc.dblk = cv.take<se_block>(n);
  oc.dorig = cv.take<int32_t>(n);
  if (own_dict) pl.phi2 = cv.take<float>(K * P);
  pl.X = cv.take<float>(n * ldV);
  pl.V = cv.take<float>(n * ldV);
  pl.R = cv.take<float>(n * ld);
  pl.D = cv.take<float>(n * ld);
  pl.rows = cv.take<float>(n * (size_t)(slots + 1) * ld);
  pl.st = cv.take<float>(2 * n);
  pl.g = cv.take<float>(2 * n * ml);
  pl.gc = pl.g ? pl.g + n * ml : nullptr;
  if (own_dict) oc.flag = cv.take<int32_t>(2);
  pl.ibuf = cv.take<int32_t>(4 + 2 * n + (slots > 0 ? n * K : 0));
  pl.deg = pl.ibuf ? pl.ibuf + 4 + n : nullptr;
  pl.cur = cv.take<int32_t>(n);
  pl.cmap = cv.take<int32_t>(n);
  if (own_dict) oc.tx = cv.take<float>(tx_const_bytes(b->M, b->N, b->n_parts) / 4);
  pl.splitk_floats = ondemand_splitk_floats(b, n_blk, tuned);
  pl.splitk = cv.take<float>(pl.splitk_floats);
  if (own_dict) oc.phi_split = cv.take<uint16_t>(2 * K * P);
  pl.Vhi = pl.Vlo = nullptr;
  if (own_dict || bf16) {
    uint16_t* vh = cv.take<uint16_t>(2 * n * ldV);
    pl.Vhi = vh;
    pl.Vlo = vh ? vh + n * ldV : nullptr;
  }
}

// Host part of a batch on demand: checks of the blocks, their order by
// decreasing iteration count (the blocks iterating at nu form a prefix),
// the device copies of the descriptors (blocks without an available sample
// marked) and the number of blocks still iterating at each nu.
struct OdBatch {
  int max_loss = 1, iters_max = 0, n_deg = 0;
  std::vector<int> it, active;
  std::vector<int32_t> order;
  std::vector<se_block> sorted;
};
static se_status plan_ondemand_batch(const se_basis* b, int n_img, int H, int W,
                                     const se_block* blocks, int n_blk, se_params prm,
                                     const int32_t* iters, OdBatch& ob) {
  if (n_img < 1 || H < 1 || W < 1) return fail(SE_EINVAL, "bad image batch");
  if (n_blk < 0 || (n_blk > 0 && !blocks)) return fail(SE_EINVAL, "bad block list");
  ob.it.assign((size_t)n_blk, 0);
  for (int i = 0; i < n_blk; ++i) {
    const se_block& bl = blocks[i];
    if (bl.img < 0 || bl.img >= n_img) return fail(SE_EINVAL, "block %d: img out of range", i);
    if (bl.lh < 1 || bl.lw < 1 || bl.ly < 0 || bl.lx < 0 || bl.ly + bl.lh > b->M ||
        bl.lx + bl.lw > b->N || bl.lt != 0 || bl.ld > 1)
      return fail(SE_EINVAL, "block %d: loss rectangle not inside the %dx%d area", i, b->M, b->N);
    ob.max_loss = std::max(ob.max_loss, bl.lh * bl.lw);
    ob.it[(size_t)i] = iters ? iters[i] : prm.iters;
    if (ob.it[(size_t)i] < 0) return fail(SE_EINVAL, "block %d: negative iteration count", i);
    ob.iters_max = std::max(ob.iters_max, ob.it[(size_t)i]);
  }
  se_status st;
  if ((st = check_loss_overlap(blocks, n_blk, H, W))) return st;
  ob.order.resize((size_t)n_blk);
  std::iota(ob.order.begin(), ob.order.end(), 0);
  std::stable_sort(ob.order.begin(), ob.order.end(), [&](int32_t x, int32_t y) {
    return ob.it[(size_t)x] > ob.it[(size_t)y];
  });
  ob.sorted.resize((size_t)n_blk);
  for (int i = 0; i < n_blk; ++i) {
    se_block v = blocks[ob.order[(size_t)i]];
    const bool none = block_without_support(v, H, W, 1, b->M, b->N);
    ob.n_deg += none;
    v.geom = none ? kBlockNoSupport : 0;
    v.ld = 1;
    ob.sorted[(size_t)i] = v;
  }
  ob.active.assign((size_t)std::max(ob.iters_max, 1), 0);
  for (int nu = 0; nu < ob.iters_max; ++nu) {
    int c = 0;
    while (c < n_blk && ob.it[(size_t)ob.order[(size_t)c]] > nu) ++c;
    ob.active[(size_t)nu] = c;
  }
  return SE_OK;
}

// (pageable sources: each copy returns once its data has been staged, so the
// vectors may go out of scope after the call)
static se_status upload_ondemand_batch(const OdBatch& ob, const OdCarve& oc, hipStream_t s) {
  hipError_t e = hipMemcpyAsync(oc.dblk, ob.sorted.data(), ob.sorted.size() * sizeof(se_block),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(oc.dorig, ob.order.data(), ob.order.size() * sizeof(int32_t),
                       hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return fail(SE_EHIP, "descriptor upload: %s", hipGetErrorString(e));
  return SE_OK;
}

// The row products' tile and split per dense range (tuner records, else the
// automatic rules; the fixed split when invariant).
static void ondemand_row_shapes(const se_basis* b, int n_blk, bool invariant, OnDemandPlan& pl) {
  const int P = b->M * b->N;
  int lo[3] = {0, 0, 0}, hi[3] = {b->K, 0, 0};
  const int nr = b->n_parts > 0 ? dense_ranges(b->K, P, b->n_parts, b->parts, lo, hi) : 1;
  for (int r = 0; r < 3; ++r) {
    pl.row_tile[r] = 0;
    pl.row_split[r] = invariant ? kSplitShape : -1;
    if (r < nr) {
      const RowTune rt = tune_lookup_rows(hi[r] - lo[r], P, n_blk);
      pl.row_tile[r] = rt.tile;
      if (!invariant) pl.row_split[r] = rt.split;
    }
  }
}

static void fill_ondemand_plan(const se_basis* b, const OdBatch& ob, const OdCarve& oc,
                               se_params prm, OnDemandPlan& pl) {
  pl.K = b->K;
  pl.M = b->M;
  pl.N = b->N;
  pl.n_blk = (int)ob.sorted.size();
  pl.phi = b->phi;
  pl.blk = oc.dblk;
  pl.orig = oc.dorig;
  pl.active = ob.active.data();
  pl.iters_max = ob.iters_max;
  pl.gamma = prm.gamma;
  pl.ldV = round4(b->M * b->N);
  pl.ld = round1024(b->K);
  pl.ldg = ob.max_loss;
  pl.n_degenerate = nullptr;
  pl.basis = b;
}

size_t se_extrapolate_ondemand_ws_bytes(const se_basis* b, int32_t n_blk, int32_t max_loss) {
  if (!b || b->K < 1 || b->M < 1 || b->N < 1 || n_blk < 0 || max_loss < 0) return 0;
  Carver cv(nullptr);
  OnDemandPlan pl{};
  OdCarve oc;
  carve_ondemand(cv, b, n_blk, max_loss, 0, true, true, false, pl, oc);
  return cv.off + 256;
}

static se_status extrapolate_ondemand(const se_basis* b, const float* w, uint8_t* images,
                                      int32_t n_img, int32_t H, int32_t W,
                                      const se_block* blocks, int32_t n_blk, se_params prm,
                                      const int32_t* iters, int32_t* sel, float* coef,
                                      float* g_loss, int32_t g_loss_ld, void* ws,
                                      size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  const bool invariant = (prm.flags & SE_INVARIANT) != 0;
  se_status st;
  if ((st = check_od_basis(b))) return st;
  if (!w || !images) return fail(SE_EINVAL, "NULL argument");
  if ((st = check_params(prm, g_loss, g_loss_ld))) return st;
  if (prm.flags & SE_ROWS_Q14) return fail(SE_EINVAL, "rows on demand take no fixed-point rows");
  OdBatch ob;
  if ((st = plan_ondemand_batch(b, n_img, H, W, blocks, n_blk, prm, iters, ob))) return st;
  if (n_blk == 0) return SE_OK;
  const size_t need = se_extrapolate_ondemand_ws_bytes(b, n_blk, ob.max_loss);
  if (!ws || ws_bytes < need) return fail(SE_ENOMEM, "workspace too small: need %zu bytes", need);
  hipStream_t s = static_cast<hipStream_t>(stream);
  Carver cv(ws);
  OnDemandPlan pl{};
  OdCarve oc;
  carve_ondemand(cv, b, n_blk, ob.max_loss, 0, true, true, false, pl, oc);
  fill_ondemand_plan(b, ob, oc, prm, pl);
  pl.slots = 0;
  pl.phi2_ready = false;
  pl.split_ready = false;
  // invariant: every product split into slices fixed by the number of
  // samples (the automatic split depends on how many blocks iterate, which
  // would change the rounding)
  pl.invariant = invariant;
  for (int r = 0; r < 3; ++r) {   // automatic shapes (the tuner's records are for plans)
    pl.row_tile[r] = 0;
    pl.row_split[r] = invariant ? kSplitShape : -1;
  }
  if (prm.flags & SE_ROWS_BF16X3) {
    pl.phi_hi = oc.phi_split;
    pl.phi_lo = oc.phi_split + (size_t)b->K * b->M * b->N;
  } else {
    pl.phi_hi = pl.phi_lo = nullptr;
    pl.Vhi = pl.Vlo = nullptr;
  }
  // declared transform parts: verified (one synchronisation of the stream),
  // then their table rows are formed as transforms
  if ((st = verify_parts(b, oc.flag, s))) return st;
  if (b->n_parts > 0 && (st = build_tx_basis(b, oc.tx, s))) return st;
  pl.tx = oc.tx;
  if ((st = upload_ondemand_batch(ob, oc, s))) return st;
  pl.w = w;
  pl.images = images;
  pl.H = H;
  pl.W = W;
  pl.sel = sel;
  pl.coef = coef;
  pl.g_loss = g_loss;
  pl.g_loss_ld = g_loss ? g_loss_ld : 0;
  if ((st = ondemand_run(pl, s))) return st;
  return degenerate_status(ob.n_deg);
}

se_status se_extrapolate_ondemand(const se_basis* b, const float* w, uint8_t* images,
                                  int32_t n_img, int32_t H, int32_t W, const se_block* blocks,
                                  int32_t n_blk, se_params prm, const int32_t* iters,
                                  int32_t* sel, float* coef, float* g_loss, int32_t g_loss_ld,
                                  void* ws, size_t ws_bytes, void* stream) {
  return extrapolate_ondemand(b, w, images, n_img, H, W, blocks, n_blk, prm, iters, sel, coef,
                              g_loss, g_loss_ld, ws, ws_bytes, stream);
}

// ---------------------------------------------------------------------------
// Prepared dictionaries and plans of rows on demand.

}  // extern "C"

struct se_od_dict {
  se_basis b{};
  uint32_t flags = 0;
  float* phi2 = nullptr;       // K x P, phi squared
  float* tx = nullptr;         // transform operands (declared parts)
  uint16_t* phi_hi = nullptr;  // split-BF16 dictionary (SE_ROWS_BF16X3)
  uint16_t* phi_lo = nullptr;
};

struct se_od_plan {
  const se_od_dict* d = nullptr;
  OdBatch ob;
  se_params prm{};
  int n_img = 0, H = 0, W = 0, slots = 0;
  OnDemandPlan pl{};
};

extern "C" {

void se_ondemand_release(se_od_dict* d) {
  if (!d) return;
  if (d->phi2) (void)hipFree(d->phi2);
  if (d->tx) (void)hipFree(d->tx);
  if (d->phi_hi) (void)hipFree(d->phi_hi);
  delete d;
}

se_status se_ondemand_prepare(const se_basis* b, uint32_t flags, se_od_dict** out,
                              void* stream) {
  g_err[0] = 0;
  if (!out) return fail(SE_EINVAL, "NULL argument");
  *out = nullptr;
  se_status st;
  if ((st = check_od_basis(b))) return st;
  if (flags & ~SE_ROWS_BF16X3) return fail(SE_EINVAL, "unknown flags 0x%x", flags);
  hipStream_t s = static_cast<hipStream_t>(stream);
  se_od_dict* d = new se_od_dict;
  d->b = *b;
  d->flags = flags;
  const size_t KP = (size_t)b->K * b->M * b->N;
  int32_t* flag = nullptr;
  auto bail = [&](se_status code) {
    if (flag) (void)hipFree(flag);
    se_ondemand_release(d);
    return code;
  };
  if (hipMalloc(reinterpret_cast<void**>(&d->phi2), KP * sizeof(float)) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&flag), 2 * sizeof(int32_t)) != hipSuccess)
    return bail(fail(SE_ENOMEM, "device allocation of %zu bytes failed", KP * sizeof(float)));
  if (b->n_parts > 0 &&
      hipMalloc(reinterpret_cast<void**>(&d->tx), tx_const_bytes(b->M, b->N, b->n_parts)) !=
          hipSuccess)
    return bail(fail(SE_ENOMEM, "device allocation of the transform operands failed"));
  if ((flags & SE_ROWS_BF16X3) &&
      hipMalloc(reinterpret_cast<void**>(&d->phi_hi), 2 * KP * sizeof(uint16_t)) != hipSuccess)
    return bail(fail(SE_ENOMEM, "device allocation of the split dictionary failed"));
  if (d->phi_hi) d->phi_lo = d->phi_hi + KP;
  launch_square(b->phi, KP, d->phi2, s);
  if ((st = check_launch("square"))) return bail(st);
  if (d->phi_hi) {
    launch_split_bf16(b->phi, KP, d->phi_hi, d->phi_lo, s);
    if ((st = check_launch("split_bf16"))) return bail(st);
  }
  if (b->n_parts > 0 && (st = build_tx_basis(b, d->tx, s))) return bail(st);
  if ((st = verify_parts(b, flag, s))) return bail(st);   // synchronises the stream
  if (hipStreamSynchronize(s) != hipSuccess)
    return bail(fail(SE_EHIP, "prepare: %s", hipGetErrorString(hipGetLastError())));
  (void)hipFree(flag);
  *out = d;
  return SE_OK;
}

size_t se_ondemand_plan_ws_bytes(const se_od_dict* d, int32_t n_blk, int32_t max_loss,
                                 int32_t row_slots) {
  if (!d || n_blk < 0 || max_loss < 0 || row_slots < 0) return 0;
  Carver cv(nullptr);
  OnDemandPlan pl{};
  OdCarve oc;
  carve_ondemand(cv, &d->b, n_blk, max_loss, std::min(row_slots, d->b.K), false,
                 (d->flags & SE_ROWS_BF16X3) != 0, true, pl, oc);
  return cv.off + 256;
}

se_status se_ondemand_plan_create(const se_od_dict* d, int32_t n_img, int32_t H, int32_t W,
                                  const se_block* blocks, int32_t n_blk, se_params prm,
                                  const int32_t* iters, int32_t row_slots, void* ws,
                                  size_t ws_bytes, void* stream, se_od_plan** out) {
  g_err[0] = 0;
  if (!out || !d) return fail(SE_EINVAL, "NULL argument");
  *out = nullptr;
  se_status st;
  if ((st = check_params(prm, nullptr, 0))) return st;
  if (prm.flags & SE_ROWS_Q14) return fail(SE_EINVAL, "rows on demand take no fixed-point rows");
  if ((prm.flags & SE_ROWS_BF16X3) && !(d->flags & SE_ROWS_BF16X3))
    return fail(SE_EINVAL, "SE_ROWS_BF16X3 needs a dictionary prepared with it");
  if (row_slots < 0) return fail(SE_EINVAL, "row_slots < 0");
  se_od_plan* p = new se_od_plan;
  if ((st = plan_ondemand_batch(&d->b, n_img, H, W, blocks, n_blk, prm, iters, p->ob))) {
    delete p;
    return st;
  }
  // rows a block can use: one per iteration at most
  p->slots = std::min(row_slots, std::min(p->ob.iters_max, d->b.K));
  const size_t need = se_ondemand_plan_ws_bytes(d, n_blk, p->ob.max_loss, p->slots);
  if (n_blk > 0 && (!ws || ws_bytes < need)) {
    delete p;
    return fail(SE_ENOMEM, "workspace too small: need %zu bytes", need);
  }
  p->d = d;
  p->prm = prm;
  p->n_img = n_img;
  p->H = H;
  p->W = W;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (n_blk > 0) {
    Carver cv(ws);
    OdCarve oc;
    const bool bf16 = (prm.flags & SE_ROWS_BF16X3) != 0;
    carve_ondemand(cv, &d->b, n_blk, p->ob.max_loss, p->slots, false,
                   (d->flags & SE_ROWS_BF16X3) != 0, true, p->pl, oc);
    fill_ondemand_plan(&d->b, p->ob, oc, prm, p->pl);
    p->pl.basis = &d->b;
    p->pl.slots = p->slots;
    p->pl.phi2 = d->phi2;
    p->pl.phi2_ready = true;
    p->pl.tx = d->tx;
    p->pl.phi_hi = bf16 ? d->phi_hi : nullptr;
    p->pl.phi_lo = bf16 ? d->phi_lo : nullptr;
    p->pl.split_ready = true;
    if (!bf16) p->pl.Vhi = p->pl.Vlo = nullptr;
    const bool invariant = (prm.flags & SE_INVARIANT) != 0;
    p->pl.invariant = invariant;
    ondemand_row_shapes(&d->b, n_blk, invariant, p->pl);
    // the descriptors, copied once (the run reads them from the device)
    if ((st = upload_ondemand_batch(p->ob, oc, s)) ||
        (hipStreamSynchronize(s) != hipSuccess &&
         (st = fail(SE_EHIP, "plan: %s", hipGetErrorString(hipGetLastError()))))) {
      delete p;
      return st;
    }
  }
  *out = p;
  return SE_OK;
}

void se_ondemand_plan_release(se_od_plan* p) { delete p; }

se_status se_ondemand_extrapolate(const se_od_dict* d, const float* w, uint8_t* images,
                                  int32_t n_img, int32_t H, int32_t W, const se_block* blocks,
                                  int32_t n_blk, se_params prm, const int32_t* iters,
                                  int32_t* sel, float* coef, float* g_loss, int32_t g_loss_ld,
                                  int32_t row_slots, void* ws, size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  if (!d || !w || !images) return fail(SE_EINVAL, "NULL argument");
  if (row_slots < 0) return fail(SE_EINVAL, "row_slots < 0");
  se_status st;
  if ((st = check_params(prm, g_loss, g_loss_ld))) return st;
  if (prm.flags & SE_ROWS_Q14) return fail(SE_EINVAL, "rows on demand take no fixed-point rows");
  if ((prm.flags & SE_ROWS_BF16X3) && !(d->flags & SE_ROWS_BF16X3))
    return fail(SE_EINVAL, "SE_ROWS_BF16X3 needs a dictionary prepared with it");
  const se_basis* b = &d->b;
  OdBatch ob;
  if ((st = plan_ondemand_batch(b, n_img, H, W, blocks, n_blk, prm, iters, ob))) return st;
  if (n_blk == 0) return SE_OK;
  const int slots = std::min(row_slots, std::min(ob.iters_max, b->K));
  const size_t need = se_ondemand_plan_ws_bytes(d, n_blk, ob.max_loss, slots);
  if (!ws || ws_bytes < need) return fail(SE_ENOMEM, "workspace too small: need %zu bytes", need);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool bf16 = (prm.flags & SE_ROWS_BF16X3) != 0;
  const bool invariant = (prm.flags & SE_INVARIANT) != 0;
  Carver cv(ws);
  OnDemandPlan pl{};
  OdCarve oc;
  carve_ondemand(cv, b, n_blk, ob.max_loss, slots, false, (d->flags & SE_ROWS_BF16X3) != 0, true,
                 pl, oc);
  fill_ondemand_plan(b, ob, oc, prm, pl);
  pl.slots = slots;
  pl.phi2 = d->phi2;
  pl.phi2_ready = true;
  pl.tx = d->tx;
  pl.phi_hi = bf16 ? d->phi_hi : nullptr;
  pl.phi_lo = bf16 ? d->phi_lo : nullptr;
  pl.split_ready = true;
  if (!bf16) pl.Vhi = pl.Vlo = nullptr;
  pl.invariant = invariant;
  for (int r = 0; r < 3; ++r) {
    pl.row_tile[r] = 0;
    pl.row_split[r] = invariant ? kSplitShape : -1;
  }
  // pageable source: the call returns once the descriptors have been staged
  if ((st = upload_ondemand_batch(ob, oc, s))) return st;
  pl.w = w;
  pl.images = images;
  pl.H = H;
  pl.W = W;
  pl.sel = sel;
  pl.coef = coef;
  pl.g_loss = g_loss;
  pl.g_loss_ld = g_loss ? g_loss_ld : 0;
  if ((st = ondemand_run(pl, s))) return st;
  return degenerate_status(ob.n_deg);
}

}  // extern "C"

namespace sefase {
// (for the tuner) the plan's dense ranges: their sizes and the pixels per atom
int ondemand_plan_dense(const se_od_plan* p, int kd[3], int* P) {
  const se_basis& b = p->d->b;
  int lo[3] = {0, 0, 0}, hi[3] = {b.K, 0, 0};
  const int nr = b.n_parts > 0 ? dense_ranges(b.K, b.M * b.N, b.n_parts, b.parts, lo, hi) : 1;
  for (int r = 0; kd && r < nr; ++r) kd[r] = hi[r] - lo[r];
  if (P) *P = b.M * b.N;
  return nr;
}
int ondemand_plan_blocks(const se_od_plan* p) { return (int)p->ob.sorted.size(); }
void ondemand_plan_set_rows(se_od_plan* p, int tile, int split) {
  const bool invariant = (p->prm.flags & SE_INVARIANT) != 0;
  for (int r = 0; r < 3; ++r) {
    p->pl.row_tile[r] = tile;
    p->pl.row_split[r] = invariant ? kSplitShape : split;
  }
}
}  // namespace sefase

extern "C" {

int32_t se_ondemand_plan_info(const se_od_plan* p, int32_t* iters_max, int32_t* max_loss,
                              int32_t* row_slots) {
  if (!p) return -1;
  if (iters_max) *iters_max = p->ob.iters_max;
  if (max_loss) *max_loss = p->ob.max_loss;
  if (row_slots) *row_slots = p->slots;
  return (int32_t)p->ob.sorted.size();
}

se_status se_ondemand_run(const se_od_plan* p, const float* w, uint8_t* images, int32_t* sel,
                          float* coef, float* g_loss, int32_t g_loss_ld, void* stream) {
  g_err[0] = 0;
  if (!p || !w || !images) return fail(SE_EINVAL, "NULL argument");
  se_status st;
  if ((st = check_params(p->prm, g_loss, g_loss_ld))) return st;
  if (g_loss && g_loss_ld < p->ob.max_loss)
    return fail(SE_EINVAL, "g_loss_ld=%d < loss size %d", g_loss_ld, p->ob.max_loss);
  if (p->ob.sorted.empty()) return SE_OK;
  OnDemandPlan pl = p->pl;
  pl.w = w;
  pl.images = images;
  pl.H = p->H;
  pl.W = p->W;
  pl.sel = sel;
  pl.coef = coef;
  pl.g_loss = g_loss;
  pl.g_loss_ld = g_loss ? g_loss_ld : 0;
  if ((st = ondemand_run(pl, static_cast<hipStream_t>(stream)))) return st;
  return degenerate_status(p->ob.n_deg);
}

se_status se_extrapolate_batch(const se_tables* t, uint8_t* images, int32_t n_img, int32_t H,
                               int32_t W, const se_block* blocks, int32_t n_blk, se_params prm,
                               int32_t* sel, float* coef, float* g_loss, int32_t g_loss_ld,
                               void* ws, size_t ws_bytes, void* stream) {
  return extrapolate(false, t, images, n_img, H, W, blocks, n_blk, prm, sel, coef, g_loss,
                     g_loss_ld, ws, ws_bytes, stream);
}

se_status se_extrapolate_batch_static(const se_tables* t, uint8_t* images, int32_t n_img,
                                      int32_t H, int32_t W, const se_block* blocks,
                                      int32_t n_blk, se_params prm, int32_t* sel, float* coef,
                                      float* g_loss, int32_t g_loss_ld, void* stream) {
  return extrapolate(false, t, images, n_img, H, W, blocks, n_blk, prm, sel, coef, g_loss,
                     g_loss_ld, nullptr, 0, stream, true);
}

se_status se_extrapolate_plain(const se_tables* t, uint8_t* images, int32_t n_img, int32_t H,
                               int32_t W, const se_block* blocks, int32_t n_blk, se_params prm,
                               int32_t* sel, float* coef, float* g_loss, int32_t g_loss_ld,
                               void* ws, size_t ws_bytes, void* stream) {
  return extrapolate(true, t, images, n_img, H, W, blocks, n_blk, prm, sel, coef, g_loss,
                     g_loss_ld, ws, ws_bytes, stream);
}

}  // extern "C"

