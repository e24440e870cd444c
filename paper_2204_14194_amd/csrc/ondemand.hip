// Fast SE when every block has its own weighting function (eq. 4 with a
// different support per block: other losses or the image border inside the
// area), so no table C can be shared (the paper notes C and D must then be
// adapted to each weighting function).  Instead of building a whole K x K
// table per block, only the rows that the iteration loop actually reads are
// formed, on demand:
//   C_b[u][k] = sum_p phi_k[p] w_b[p] phi_u[p]        (eq. 16, row u)
// For a group of blocks sharing the dictionary that advance one iteration at
// a time, the rows of all blocks are one matrix product on the matrix cores:
//   rows = Phi V^T,  V[b][p] = w_b[p] phi_{u_b}[p].
// Likewise C_b[k][k] = sum_p phi_k[p]^2 w_b[p] (the per-block D_b, eq. 17)
// and the initial projections R_b^(0) = Phi (w_b s_b) (eq. 12) are products
// with the same dictionary.
//
// The dense row products may take split-BF16 operands (three BF16 matrix-core
// products, FP32 accumulation): the dictionary split once per call, the V
// rows split where they are written.
//
// Per iteration a workgroup per block applies the previous update (eq. 20,
// in units of D_b), selects the next atom (eq. 18), records c (eq. 19),
// updates the model over the loss (eq. 9) and writes its V row.  All state
// lives in device memory between the launches.  Blocks are processed in
// decreasing order of their iteration counts, so the blocks still running at
// iteration nu form a prefix and each launch covers only that prefix.
#include "argmax.h"
#include "bf16.h"
#include "se_internal.h"

namespace sefase {

constexpr int kOdThreads = 256;

// X[b][p] = w_b[p] s_b[p] (the weighted signal, eq. 12); V rows reuse the
// same layout.
__global__ void k_od_gather(const uint8_t* __restrict__ images, int H, int W,
                            const DevBlock* __restrict__ blk, int n_blk, int M, int N,
                            const float* __restrict__ w, const int32_t* __restrict__ orig,
                            float* __restrict__ X, int ldX) {
  const int b = blockIdx.y;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int P = M * N;
  if (b >= n_blk || p >= P) return;
  const DevBlock d = blk[b];
  const int m = p / N, n = p - m * N;
  const int y = d.y0 + m, x = d.x0 + n;
  float v = 0.0f;
  if (y >= 0 && y < H && x >= 0 && x < W)
    v = w[(size_t)orig[b] * P + p] * (float)images[(size_t)d.img * H * W + (size_t)y * W + x];
  X[(size_t)b * ldX + p] = v;
}

// V[b][p] = w_b[p] (the weights as rows of the diagonal product)
__global__ void k_od_gather_w(const float* __restrict__ w, const int32_t* __restrict__ orig,
                              int n_blk, int P, float* __restrict__ V, int ldV) {
  const int b = blockIdx.y;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_blk || p >= P) return;
  V[(size_t)b * ldV + p] = w[(size_t)orig[b] * P + p];
}

__global__ void k_fill0(float* __restrict__ a, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0f;
}

__global__ void k_square(const float* __restrict__ phi, size_t n, float* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = phi[i] * phi[i];
}

// D_b = 1/sqrt(C_b[k][k]) (0 for a non-positive diagonal); R~ = D_b R^(0).
// Dd holds the diagonal on entry and D_b on exit.
__global__ void k_od_init(float* __restrict__ Dd, float* __restrict__ R, int n_blk, int ld) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)n_blk * ld) return;
  const float dd = Dd[i];
  const float D = dd > 0.0f ? 1.0f / sqrtf(dd) : 0.0f;
  Dd[i] = D;
  R[i] = D * R[i];
}

struct OdArgs {
  float* R;            // n_blk x ld, R~ = D_b R (units of D_b)
  const float* D;      // n_blk x ld
  const float* rows;   // n_blk x (slots + 1) rows of ld: the row cache
  int slots;           // cached rows per block; row `slots` is recomputed on every use
  int32_t* slot_of;    // n_blk x K: 1 + cache row of atom k's row, 0 if none (NULL: slots 0)
  int32_t* nslot;      // n_blk: cache rows in use
  int32_t* cur;        // n_blk: cache row of the last selection's row
  int32_t* cnt;        // 2: rows requested in this iteration (by parity)
  int32_t* cmap;       // requested row i -> its row in the cache
  int nxt;             // blocks that iterate again (a prefix)
  float* V;            // rows requested in this iteration: w_b phi_u (compact)
  uint16_t* Vhi;       // optional split copy of V (split-BF16 row products)
  uint16_t* Vlo;
  int ld, ldV;
  const float* phi;    // K x P
  const float* w;      // original-order blocks x P
  const DevBlock* blk; // sorted by decreasing iteration count
  const int32_t* orig; // sorted position -> caller's block index
  float* st;           // n_blk x 2: t_prev, D_u_prev (per block)
  float* g;            // n_blk x ldg model over the loss (sorted order)
  float* gc;           // Kahan compensation
  int ldg;
  int K, M, N;
  int nu, iters_max;
  float gamma;
  int32_t* sel;        // optional, caller order, stride iters_max
  float* coef;         // optional
  int32_t* deg;        // n_blk: 1 for a block with nothing to extrapolate from
  int32_t* n_degenerate;   // optional device counter of such blocks
};

__global__ __launch_bounds__(kOdThreads) void k_od_step(OdArgs a) {
  const int b = blockIdx.x;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int K = a.K, P = a.M * a.N;
  float* R = a.R + (size_t)b * a.ld;
  const float* D = a.D + (size_t)b * a.ld;
  const bool upd = a.nu > 0;
  const int ob = a.orig[b];
  // the request counter of the next iteration starts at 0 (the products of
  // the previous iteration, its last readers, have completed)
  if (b == 0 && t == 0) a.cnt[(a.nu + 1) & 1] = 0;
  // a block with nothing to extrapolate from (no available sample, marked by
  // the host, or every atom of zero weighted norm: D_b = 0 and R~ = 0
  // everywhere) reports sel = -1 and a zero coefficient in every iteration
  if (a.nu == 0) {
    bool deg = (a.blk[b].geom & kBlockNoSupport) != 0;
    if (!deg) {
      bool nz = false;
      for (int k = t; k < K; k += kOdThreads) nz = nz || R[k] != 0.0f || D[k] != 0.0f;
      deg = !any_in_workgroup<kOdThreads / 64>(nz);
    }
    if (t == 0) {
      a.deg[b] = deg;
      if (deg && a.n_degenerate) atomicAdd(a.n_degenerate, 1);
    }
    if (deg) {
      if (t == 0 && a.sel) a.sel[(size_t)ob * a.iters_max] = -1;
      if (t == 0 && a.coef) a.coef[(size_t)ob * a.iters_max] = 0.0f;
      return;
    }
  } else if (a.deg[b]) {
    if (t == 0 && a.sel) a.sel[(size_t)ob * a.iters_max + a.nu] = -1;
    if (t == 0 && a.coef) a.coef[(size_t)ob * a.iters_max + a.nu] = 0.0f;
    return;
  }
  float sc = 0.0f;
  if (upd) sc = a.st[2 * b] * a.st[2 * b + 1];   // gamma R~_u D_u: the eq. 20 factor
  // the row C_b[u_prev][:] (cached, or formed after the previous launch)
  const float* rows = a.rows + ((size_t)b * (a.slots + 1) + (upd ? a.cur[b] : 0)) * a.ld;
  // update with the previous row, then find this lane's first strict maximum
  // (and its D, so the winner's D_u needs no further load)
  float bv = 0.0f, bd = 0.0f;
  int bi = 0x7fffffff;
  const int nj = a.ld / (4 * kOdThreads);
  for (int j = 0; j < nj; ++j) {
    const int k0 = 4 * (j * kOdThreads + t);
    if (k0 >= K) break;   // the padding (always 0) is neither updated nor a candidate
    float4 r = *reinterpret_cast<const float4*>(R + k0);
    const float4 d = *reinterpret_cast<const float4*>(D + k0);
    if (upd) {
      float4 c = *reinterpret_cast<const float4*>(rows + k0);
      if (k0 + 4 > K) {   // row entries past K are never written
        c.y = k0 + 1 < K ? c.y : 0.0f;
        c.z = k0 + 2 < K ? c.z : 0.0f;
        c.w = 0.0f;
      }
      r.x = fmaf(-sc * d.x, c.x, r.x);
      r.y = fmaf(-sc * d.y, c.y, r.y);
      r.z = fmaf(-sc * d.z, c.z, r.z);
      r.w = fmaf(-sc * d.w, c.w, r.w);
      *reinterpret_cast<float4*>(R + k0) = r;
    }
    if (fabsf(r.x) > fabsf(bv)) { bv = r.x; bi = k0; bd = d.x; }
    if (fabsf(r.y) > fabsf(bv)) { bv = r.y; bi = k0 + 1; bd = d.y; }
    if (fabsf(r.z) > fabsf(bv)) { bv = r.z; bi = k0 + 2; bd = d.z; }
    if (fabsf(r.w) > fabsf(bv)) { bv = r.w; bi = k0 + 3; bd = d.w; }
  }
  const uint64_t mine = make_key(bv, bi == 0x7fffffff ? 0 : bi);
  uint64_t key = wave_max_key((uint32_t)(mine >> 32), (uint32_t)mine);
  // the D of the wave's winner (the lane whose key is the maximum; keys of
  // different atoms differ, and with every score 0 the coefficient is 0
  // whatever D is taken)
  const int wl = (int)__builtin_ctzll(__builtin_amdgcn_ballot_w64(mine == key));
  const float wd = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(bd), wl));
  __shared__ uint64_t s_key[kOdThreads / 64];
  __shared__ float s_d[kOdThreads / 64];
  if (lane == 0) {
    s_key[wave] = key;
    s_d[wave] = wd;
  }
  __syncthreads();
  key = s_key[0];
  float Du = s_d[0];
#pragma unroll
  for (int i = 1; i < kOdThreads / 64; ++i)
    if (s_key[i] > key) {
      key = s_key[i];
      Du = s_d[i];
    }
  int u;
  float rv;
  decode_key(key, K, u, rv);
  const float tc = a.gamma * rv;          // coefficient of the unit-norm atom
  const float c = tc * Du;                // eq. 19
  if (t == 0) {
    a.st[2 * b] = tc;
    a.st[2 * b + 1] = Du;
    if (a.sel) a.sel[(size_t)ob * a.iters_max + a.nu] = u;
    if (a.coef) a.coef[(size_t)ob * a.iters_max + a.nu] = c;
  }
  // the row C_b[u][:] for the next iteration: a cached row, or a request
  // (w_b phi_u as a compact row of V) for the products after this launch;
  // decided by the last wave while the first ones update the model
  const bool more = b < a.nxt;
  __shared__ int s_req;
  if (more && t == kOdThreads - 64) {
    int32_t* so = a.slot_of ? a.slot_of + (size_t)b * K + u : nullptr;
    const int have = so ? *so : 0;
    int row = a.slots;                     // the row recomputed on every use
    int req = -1;
    if (have > 0) {
      row = have - 1;
    } else {
      if (so && a.nslot[b] < a.slots) {
        row = a.nslot[b]++;
        *so = row + 1;
      }
      req = atomicAdd(a.cnt + (a.nu & 1), 1);
      a.cmap[req] = b * (a.slots + 1) + row;
    }
    a.cur[b] = row;
    s_req = req;
  }
  // model over the loss (eq. 9), compensated
  const DevBlock d = a.blk[b];
  const float* prow = a.phi + (size_t)u * P;
  const int nloss = d.lh * d.lw;
  for (int q = t; q < nloss; q += kOdThreads) {
    const int my = q / d.lw, mx = q - my * d.lw;
    const float pv = prow[(d.ly + my) * a.N + d.lx + mx];
    float* gp = a.g + (size_t)b * a.ldg + q;
    float* cp = a.gc + (size_t)b * a.ldg + q;
    const float y = fmaf(c, pv, -*cp);
    const float s = *gp + y;
    *cp = (s - *gp) - y;
    *gp = s;
  }
  if (!more) return;
  __syncthreads();
  const int req = s_req;
  if (req < 0) return;
  const float* wb = a.w + (size_t)ob * P;
  float* V = a.V + (size_t)req * a.ldV;
  if (a.Vhi) {
    uint16_t* Vh = a.Vhi + (size_t)req * a.ldV;
    uint16_t* Vl = a.Vlo + (size_t)req * a.ldV;
    for (int p = t; p < P; p += kOdThreads) {
      const float v = wb[p] * prow[p];
      uint16_t h, l;
      bf16_split(v, h, l);
      V[p] = v;
      Vh[p] = h;
      Vl[p] = l;
    }
  } else {
    for (int p = t; p < P; p += kOdThreads) V[p] = wb[p] * prow[p];
  }
}

// paste the model into the image and (optionally) report it
__global__ void k_od_finish(const DevBlock* __restrict__ blk, const int32_t* __restrict__ orig,
                            const float* __restrict__ g, int ldg, uint8_t* __restrict__ images,
                            int H, int W, float* __restrict__ g_loss, int g_loss_ld,
                            const int32_t* __restrict__ deg) {
  const int b = blockIdx.x;
  const DevBlock d = blk[b];
  const int nloss = d.lh * d.lw;
  const int ob = orig[b];
  const bool none = deg[b] != 0;           // no model: the loss is left as it is
  for (int q = threadIdx.x; q < nloss; q += blockDim.x) {
    const float v = none ? 0.0f : g[(size_t)b * ldg + q];
    if (g_loss && q < g_loss_ld) g_loss[(size_t)ob * g_loss_ld + q] = v;
    if (none) continue;
    const int my = q / d.lw, mx = q - my * d.lw;
    const int y = d.y0 + d.ly + my, x = d.x0 + d.lx + mx;
    if (y >= 0 && y < H && x >= 0 && x < W)
      images[(size_t)d.img * H * W + (size_t)y * W + x] =
          (uint8_t)fminf(fmaxf(rintf(v), 0.0f), 255.0f);
  }
}

// ---------------------------------------------------------------------------
__global__ void k_fill0_i32(int32_t* __restrict__ a, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0;
}

void launch_square(const float* phi, size_t n, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_square, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, phi, n, out);
}

// Only kernel launches, whose shapes depend on the plan alone (no copy, no
// fill through the runtime, no synchronisation): a run can be captured in a
// graph and replayed.
se_status ondemand_run(const OnDemandPlan& pl, hipStream_t s) {
  se_status st;
  const int K = pl.K, P = pl.M * pl.N, n = pl.n_blk;
  // model accumulators start at 0 (g and gc are adjacent); request counters,
  // rows in use and the atom -> cached row map too
  hipLaunchKernelGGL(k_fill0, dim3((unsigned)(((size_t)2 * n * pl.ldg + 255) / 256)), dim3(256), 0,
                     s, pl.g, (size_t)2 * n * pl.ldg);
  if ((st = check_launch("fill0"))) return st;
  const size_t ni = 4 + 2 * (size_t)n + (pl.slots > 0 ? (size_t)n * K : 0);
  hipLaunchKernelGGL(k_fill0_i32, dim3((unsigned)((ni + 255) / 256)), dim3(256), 0, s, pl.ibuf, ni);
  if ((st = check_launch("fill0_i32"))) return st;
  // dictionary squared (for the per-block diagonal), unless prepared
  if (!pl.phi2_ready) {
    hipLaunchKernelGGL(k_square, dim3((unsigned)(((size_t)K * P + 255) / 256)), dim3(256), 0, s,
                       pl.phi, (size_t)K * P, pl.phi2);
    if ((st = check_launch("square"))) return st;
  }
  // weighted signal and weights as row blocks of the products
  hipLaunchKernelGGL(k_od_gather, dim3((P + 255) / 256, n), dim3(256), 0, s, pl.images, pl.H,
                     pl.W, pl.blk, n, pl.M, pl.N, pl.w, pl.orig, pl.X, pl.ldV);
  if ((st = check_launch("od_gather"))) return st;
  hipLaunchKernelGGL(k_od_gather_w, dim3((P + 255) / 256, n), dim3(256), 0, s, pl.w, pl.orig, n,
                     P, pl.V, pl.ldV);
  if ((st = check_launch("od_gather_w"))) return st;
  const int split_rule = pl.invariant ? kSplitShape : -1;
  if ((st = gemm_project_f32(pl.phi2, P, K, pl.V, pl.ldV, n, P, pl.D, pl.ld, 0, s, true,
                             pl.splitk, pl.splitk_floats, split_rule)))
    return st;
  if ((st = gemm_project_f32(pl.phi, P, K, pl.X, pl.ldV, n, P, pl.R, pl.ld, 0, s, true, pl.splitk,
                             pl.splitk_floats, split_rule)))
    return st;
  hipLaunchKernelGGL(k_od_init, dim3((unsigned)(((size_t)n * pl.ld + 255) / 256)), dim3(256), 0,
                     s, pl.D, pl.R, n, pl.ld);
  if ((st = check_launch("od_init"))) return st;
  OdArgs a;
  a.R = pl.R;
  a.D = pl.D;
  a.rows = pl.rows;
  a.slots = pl.slots;
  a.cnt = pl.ibuf;
  a.nslot = pl.ibuf + 4;
  a.slot_of = pl.slots > 0 ? pl.ibuf + 4 + 2 * (size_t)n : nullptr;
  a.cur = pl.cur;
  a.cmap = pl.cmap;
  a.V = pl.V;
  a.ld = pl.ld;
  a.ldV = pl.ldV;
  a.phi = pl.phi;
  a.w = pl.w;
  a.blk = pl.blk;
  a.orig = pl.orig;
  a.st = pl.st;
  a.g = pl.g;
  a.gc = pl.gc;
  a.ldg = pl.ldg;
  a.K = K;
  a.M = pl.M;
  a.N = pl.N;
  a.iters_max = pl.iters_max;
  a.gamma = pl.gamma;
  a.sel = pl.sel;
  a.coef = pl.coef;
  a.deg = pl.deg;
  a.n_degenerate = pl.n_degenerate;
  // atoms whose rows come from the dictionary product (all of them without
  // transform parts)
  const se_basis* bs = pl.basis;
  const bool tx = bs && bs->n_parts > 0;
  int lo[3] = {0, 0, 0}, hi[3] = {K, 0, 0};
  const int nr = tx ? dense_ranges(K, pl.M * pl.N, bs->n_parts, bs->parts, lo, hi) : 1;
  const bool split = pl.phi_hi != nullptr && nr > 0;   // no dense atoms: nothing to split
  if (split && !pl.split_ready) {
    launch_split_bf16(pl.phi, (size_t)K * P, pl.phi_hi, pl.phi_lo, s);
    if ((st = check_launch("split_bf16"))) return st;
  }
  a.Vhi = split ? pl.Vhi : nullptr;
  a.Vlo = split ? pl.Vlo : nullptr;
  const size_t rows_ld = (size_t)pl.ld;
  for (int nu = 0; nu < pl.iters_max; ++nu) {
    const int act = pl.active[nu];        // blocks still iterating at nu (a prefix)
    if (act <= 0) break;
    const int nxt = nu + 1 < pl.iters_max ? pl.active[nu + 1] : 0;
    a.nu = nu;
    a.nxt = nxt;
    hipLaunchKernelGGL(k_od_step, dim3(act), dim3(kOdThreads), 0, s, a);
    if ((st = check_launch("od_step"))) return st;
    if (nxt <= 0) continue;
    // rows C_b[u_b][:] requested by the blocks that iterate again (at most
    // nxt, counted on the device): transforms of w_b phi_u for the parts, a
    // product with the dictionary for the rest, each written to its row of
    // the cache
    const int32_t* cnt = pl.ibuf + (nu & 1);
    if (tx && (st = rows_tx(bs, pl.tx, pl.V, pl.ldV, nxt, pl.rows, (int)rows_ld, s, cnt,
                            pl.cmap)))
      return st;
    for (int r = 0; r < nr; ++r) {
      st = split ? gemm_rows_bf16x3(pl.phi_hi + (size_t)lo[r] * P, pl.phi_lo + (size_t)lo[r] * P,
                                    P, hi[r] - lo[r], pl.Vhi, pl.Vlo, pl.ldV, nxt, cnt, pl.cmap, P,
                                    pl.rows + lo[r], (int)rows_ld, pl.row_tile[r], s)
                 : gemm_rows_f32(pl.phi + (size_t)lo[r] * P, P, hi[r] - lo[r], pl.V, pl.ldV, nxt,
                                 cnt, pl.cmap, P, pl.rows + lo[r], (int)rows_ld, pl.row_tile[r],
                                 pl.row_split[r], s, pl.splitk, pl.splitk_floats);
      if (st) return st;
    }
  }
  hipLaunchKernelGGL(k_od_finish, dim3(n), dim3(256), 0, s, pl.blk, pl.orig, pl.g, pl.ldg,
                     pl.images, pl.H, pl.W, pl.g_loss, pl.g_loss_ld, pl.deg);
  return check_launch("od_finish");
}

}  // namespace sefase
