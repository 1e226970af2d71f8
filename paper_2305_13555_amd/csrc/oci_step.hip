// One-cell inversion hot path: per-step constant, the block-Jacobi iteration
// and the end of step (Sec. "One-Cell Inversion (OCI)").
//
// For every cell j of region r the iteration solves (A - S) Psi_j = c_j with
// the incident fluxes of c^+ / c^- taken from the neighbours' previous
// iterate.  c_j is linear in (incident fluxes, psi_{k-1/2}, Q), so with the
// operator formed at setup (rows of (A - S)^{-1} applied to those columns)
// each iteration of a whole region is one GEMM over its cells:
//
//   [out_j ; phi_j]^(l+1) = G_r inc_j^(l) + [g_j ; h_j]              (hot)
//   [g_j ; h_j]           = P_r psi_{k-1/2,j} + p_r                  (once per step)
//   psi_{k+1/2,j}         = E_r [inc_j^(L-1) ; psi_{k-1/2,j}] + e_r  (end of step)
//
// which is the same iteration as solving every cell's dense system with its
// LU factors, in a different association of the same products.  G_r is
// (2N+4) x 2N, applied with v_mfma_f64_16x16x4f64 to a 16-cell tile: the
// A operand is the tile's incident fluxes (one cell per MFMA row), gathered
// from the outgoing rows of the neighbouring cells staged in LDS; the B
// operand is the operator, packed in fragment order, L2-resident and shared
// by every tile of the region.
//
// Each iteration is one launch with no device-scope synchronisation inside:
// every work-group first re-derives the stopping decision for the previous
// iterate from the per-tile residual records that launch left behind (they
// are visible because the launches are ordered), and exits at once if the
// step is decided; otherwise it computes its tile and leaves its own record.
// The work-group that takes a decision first also writes it to the step
// control block, which later launches read.
#include "oci_kernels.h"

namespace ocik {

// Work-group index -> tile: consecutive tiles go to the same XCD (work-groups
// are dispatched round-robin over the 8 XCDs), so a region's operator is
// read into few L2s and neighbouring tiles share an L2.  The grid has
// 8*ceil(ntiles/8) work-groups, on which this map is a bijection; the
// surplus ones get -1 and exit.
__device__ __forceinline__ int tile_of_block(int b, int ntiles) {
  const int nx = 8;
  const int per = (ntiles + nx - 1) / nx;
  const int t = (b % nx) * per + b / nx;
  return t < ntiles ? t : -1;
}

// A block of consecutive rows (row length K doubles, K even) copied from
// global memory into LDS rows of pitch P; LDS rows rows .. cap-1 are zeroed.
struct RowBlock {
  const double *src;   // first row in global memory
  double *dst;         // first LDS row
  int rows;            // rows to copy
  int cap;             // LDS rows owned by the block (rows .. cap-1 are zeroed)
};

// Staged copy: the first batch of every thread's elements is held in
// registers between issue_copy (loads) and finish_copy (LDS stores and any
// further batches), so the loads can be issued early.
constexpr int kCopyBatch = 4;
struct CopyRegs {
  double2 v[kCopyBatch];
};

__device__ __forceinline__ int copy_total(const RowBlock *blk, int nblk, int h, int *off1) {
  const int n0 = blk[0].cap * h;
  *off1 = n0;
  return nblk > 1 ? n0 + blk[1].cap * h : n0;
}

__device__ __forceinline__ double2 copy_load(const RowBlock *blk, int nblk, int h, int off1,
                                             int i) {
  const int b = (nblk > 1 && i >= off1) ? 1 : 0;
  const int li = b ? i - off1 : i;
  if (li / h < blk[b].rows) return reinterpret_cast<const double2 *>(blk[b].src)[li];
  return make_double2(0.0, 0.0);
}

__device__ __forceinline__ void copy_store(const RowBlock *blk, int nblk, int h, int off1, int P,
                                           int i, double2 v) {
  const int b = (nblk > 1 && i >= off1) ? 1 : 0;
  const int li = b ? i - off1 : i;
  const int r = li / h, c2 = li - r * h;
  *reinterpret_cast<double2 *>(blk[b].dst + r * P + 2 * c2) = v;
}

__device__ inline void issue_copy(CopyRegs &cr, const RowBlock *blk, int nblk, int K) {
  const int h = K / 2;
  int off1;
  const int total = copy_total(blk, nblk, h, &off1);
#pragma unroll
  for (int q = 0; q < kCopyBatch; ++q) {
    const int i = threadIdx.x + q * blockDim.x;
    cr.v[q] = i < total ? copy_load(blk, nblk, h, off1, i) : make_double2(0.0, 0.0);
  }
}

__device__ inline void finish_copy(const CopyRegs &cr, const RowBlock *blk, int nblk, int K,
                                   int P) {
  const int h = K / 2;
  int off1;
  const int total = copy_total(blk, nblk, h, &off1);
#pragma unroll
  for (int q = 0; q < kCopyBatch; ++q) {
    const int i = threadIdx.x + q * blockDim.x;
    if (i < total) copy_store(blk, nblk, h, off1, P, i, cr.v[q]);
  }
  for (int base = threadIdx.x + kCopyBatch * blockDim.x; base < total;
       base += kCopyBatch * blockDim.x) {
    double2 v[kCopyBatch];
#pragma unroll
    for (int q = 0; q < kCopyBatch; ++q) {
      const int i = base + q * blockDim.x;
      v[q] = i < total ? copy_load(blk, nblk, h, off1, i) : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int q = 0; q < kCopyBatch; ++q) {
      const int i = base + q * blockDim.x;
      if (i < total) copy_store(blk, nblk, h, off1, P, i, v[q]);
    }
  }
}

// Copy blocks of consecutive rows into LDS (one memory round trip per
// kCopyBatch elements per thread).  No barrier inside.
__device__ inline void copy_blocks_to_lds(const RowBlock *blk, int nblk, int K, int P) {
  CopyRegs cr;
  issue_copy(cr, blk, nblk, K);
  finish_copy(cr, blk, nblk, K, P);
}

// Reflecting edges in a staged neighbour block: the ghost row takes the
// boundary cell's mirror-angle values.  Call after the staged rows are
// visible (barrier); ends with a barrier.
__device__ inline void reflect_ghosts(double *lds, int P, const TileDev &t, int N, int J, int bcl,
                                      int bcr) {
  const int K = 2 * N;
  if (t.c0 == 0 && bcl == kBcReflect) {
    // entering at x = 0 in angle m (mu > 0) = leaving in angle N-1-m
    for (int i = N + threadIdx.x; i < K; i += blockDim.x) {
      const int m = i >> 1, tl = i & 1;
      lds[i] = lds[P + 2 * (N - 1 - m) + tl];
    }
  }
  if (t.c0 + t.nc == J && bcr == kBcReflect) {
    const int rg = t.nc + 1;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
      const int m = i >> 1, tl = i & 1;
      lds[rg * P + i] = lds[(rg - 1) * P + 2 * (N - 1 - m) + tl];
    }
  }
  __syncthreads();
}

// The outgoing rows of cells c0-1 .. c0+nc (ghosted rows c0 .. c0+nc+1) as
// a copy block into LDS rows 0 .. 17.
__device__ __forceinline__ RowBlock neighbour_block(double *lds, const double *src,
                                                    const TileDev &t, int K) {
  return RowBlock{src + (size_t)t.c0 * K, lds, t.nc + 2, kTileCells + 2};
}

// Rows c0 .. c0+nc-1 of a [J][K] array as a copy block into LDS rows 0..15.
__device__ __forceinline__ RowBlock own_block(double *lds, const double *src, const TileDev &t,
                                              int K) {
  return RowBlock{src + (size_t)t.c0 * K, lds, t.nc, kTileCells};
}

// Operator fragments for k-steps base .. base+CH-1 of one row tile (zero past KS).
template <int CH>
__device__ __forceinline__ void load_frags(double (&f)[CH], const double *Fr, int base, int KS) {
#pragma unroll
  for (int i = 0; i < CH; ++i) f[i] = (base + i < KS) ? Fr[(size_t)(base + i) * 64] : 0.0;
}

// acc += A(16 cells x 4CH) * B(4CH x 16 rows) for one chunk; aload(ks) gives
// this lane's A element of k-step ks.
template <int CH, typename ALoad>
__device__ __forceinline__ void mma_chunk(d4 &acc, const double (&f)[CH], int base, int KS,
                                          ALoad aload) {
#pragma unroll
  for (int i = 0; i < CH; ++i)
    if (base + i < KS) acc = mfma16x16x4(aload(base + i), f[i], acc);
}

// One row tile: chunks of CH k-steps; the first chunk's fragments may come
// preloaded.
template <int CH, typename ALoad>
__device__ __forceinline__ d4 mma_rowtile(const double *Fr, int KS, bool first_loaded,
                                          const double (&f0)[CH], ALoad aload) {
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int base = 0; base < KS; base += CH) {
    double f[CH];
    if (first_loaded && base == 0) {
#pragma unroll
      for (int i = 0; i < CH; ++i) f[i] = f0[i];
    } else {
      load_frags<CH>(f, Fr, base, KS);
    }
    mma_chunk<CH>(acc, f, base, KS, aload);
  }
  return acc;
}

// ---------------------------------------------------------------------------
// Tile routines
// ---------------------------------------------------------------------------

// gh rows of a tile: gh_j = P_r psi_{k-1/2,j} + p_r.
template <int CH>
__device__ inline void tile_begin(const StepArgs &a, const TileDev &t, const double *psi_prev,
                                  double *lds) {
  const int N = a.N, K = 2 * N, P = K + 2, KS = K / 4;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, W = blockDim.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const double *F = a.frag_pv + (size_t)t.region * a.frag_pv_stride + lane;
  const double *cp = a.c_pv + (size_t)t.region * a.c_pv_stride;
  const int ghp = a.Mt * 16;
  double f0[CH];
  if (wave < a.Mt) load_frags<CH>(f0, F + (size_t)wave * KS * 64, 0, KS);
  const RowBlock blk[1] = {own_block(lds, psi_prev, t, K)};
  copy_blocks_to_lds(blk, 1, K, P);
  __syncthreads();
  const double *arow = lds + col * P + kq;
  auto aload = [&](int ks) { return arow[ks * 4]; };
  for (int rt = wave; rt < a.Mt; rt += W) {
    const d4 acc = mma_rowtile<CH>(F + (size_t)rt * KS * 64, KS, rt == wave, f0, aload);
    const int row = rt * 16 + col;
    const double cv = cp[row];
    for (int i = 0; i < 4; ++i) {
      const int cl = kq + 4 * i;
      if (cl < t.nc) a.gh[(size_t)(t.c0 + cl) * ghp + row] = acc[i] + cv;
    }
  }
}

// One OCI iteration of a tile, in two phases so that the caller can take
// the stopping decision between them.  iterate_prefetch issues every load
// that does not depend on LDS: the first operator chunk of the wave's first
// row tile and that row tile's constants, the scalar-flux constants and old
// values, and the neighbour rows and scalar-flux operator rows (staged into
// LDS by iterate_compute).  iterate_compute runs the GEMM for the 2N outgoing
// rows on MFMA, the 4 scalar-flux rows as dot products split over W threads
// per (cell, component), and writes the tile's residual record.
template <int CH>
struct IterPrefetch {
  double f0[CH], gv[4];
  double hv, po;   // scalar-flux constant and previous value of this thread's (cell, component)
  CopyRegs cr;
};

template <int CH>
__device__ __forceinline__ void iterate_blocks(RowBlock (&blk)[2], const StepArgs &a,
                                               const TileDev &t, const double *src, double *lds) {
  const int K = 2 * a.N;
  blk[0] = neighbour_block(lds, src, t, K);
  blk[1] = RowBlock{a.hphi + (size_t)t.region * a.hphi_stride, lds + (kTileCells + 2) * (K + 2), 4,
                    4};
}

template <int CH>
__device__ inline void iterate_prefetch(IterPrefetch<CH> &pf, const StepArgs &a, const TileDev &t,
                                        const double *src, const double *phi_old, double *lds) {
  const int N = a.N, K = 2 * N, KS = K / 4;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, W = blockDim.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const double *F = a.frag_it + (size_t)t.region * a.frag_it_stride + lane;
  const int ghp = a.Mt * 16;
  const int row0 = wave * 16 + col;
  if (wave < a.Mto) load_frags<CH>(pf.f0, F + (size_t)wave * KS * 64, 0, KS);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int cl = kq + 4 * i;
    const bool ok = wave < a.Mto && row0 < K && cl < t.nc;
    pf.gv[i] = ok ? a.gh[(size_t)(t.c0 + cl) * ghp + row0] : 0.0;
  }
  const int pair = threadIdx.x / W, cl = pair >> 2, comp = pair & 3;
  const bool pok = cl < t.nc;
  pf.hv = pok ? a.gh[(size_t)(t.c0 + cl) * ghp + K + comp] : 0.0;
  pf.po = pok ? phi_old[(size_t)(t.c0 + cl) * 4 + comp] : 0.0;
  RowBlock blk[2];
  iterate_blocks<CH>(blk, a, t, src, lds);
  issue_copy(pf.cr, blk, 2, K);
}

// Writes the tile's residual record (rec); ends with a barrier.
template <int CH>
__device__ inline void iterate_compute(const IterPrefetch<CH> &pf, const StepArgs &a,
                                       const TileDev &t, const double *src, double *dst,
                                       double *phi_new, double *lds, double *scratch,
                                       double2 *rec) {
  const int N = a.N, K = 2 * N, P = K + 2, KS = K / 4;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, W = blockDim.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const double *F = a.frag_it + (size_t)t.region * a.frag_it_stride + lane;
  const int ghp = a.Mt * 16;
  {
    RowBlock blk[2];
    iterate_blocks<CH>(blk, a, t, src, lds);
    finish_copy(pf.cr, blk, 2, K, P);
  }
  __syncthreads();
  reflect_ghosts(lds, P, t, N, a.J, a.bcl, a.bcr);
  // incident flux of cell c, entry k: k < N from the right neighbour
  // (LDS row c+2), k >= N from the left neighbour (LDS row c)
  auto aload = [&](int ks) {
    const int k = ks * 4 + kq;
    return lds[(k < N ? col + 2 : col) * P + k];
  };
  for (int rt = wave; rt < a.Mto; rt += W) {
    const d4 acc = mma_rowtile<CH>(F + (size_t)rt * KS * 64, KS, rt == wave, pf.f0, aload);
    const int row = rt * 16 + col;      // outgoing row of this lane
    if (row < K) {
      for (int i = 0; i < 4; ++i) {
        const int cl = kq + 4 * i;      // cell of element i
        if (cl >= t.nc) continue;
        const int cell = t.c0 + cl;
        const double g = rt == wave ? pf.gv[i] : a.gh[(size_t)cell * ghp + row];
        dst[(size_t)(cell + 1) * K + row] = acc[i] + g;
      }
    }
  }
  // scalar flux: W threads per (cell, component), each a K/W slice of the
  // dot product with the scalar-flux operator row (LDS rows 18..21)
  const int q = threadIdx.x % W, pair = threadIdx.x / W, cl = pair >> 2, comp = pair & 3;
  const int T = K / W;
  const double *hrow = lds + (kTileCells + 2 + comp) * P;
  double s = 0.0;
  for (int kk = 0; kk < T; ++kk) {
    const int k = q * T + kk;
    s += hrow[k] * lds[(k < N ? cl + 2 : cl) * P + k];
  }
  for (int o = 1; o < W; o <<= 1) s += __shfl_xor(s, o, kWave);
  double dphi = 0.0, fphi = 0.0;
  if (q == 0 && cl < t.nc) {
    const double v = s + pf.hv;
    phi_new[(size_t)(t.c0 + cl) * 4 + comp] = v;
    dphi = isfinite(v) ? fabs(v - pf.po) : __builtin_nan("");
    fphi = fabs(v);
  }
  dphi = wave_nan_max(dphi);
  fphi = wave_max(fphi);
  if (lane == 0) {
    scratch[wave * 2 + 0] = dphi;
    scratch[wave * 2 + 1] = fphi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < W; ++w) {
      dphi = nan_max(dphi, scratch[w * 2 + 0]);
      fphi = fmax(fphi, scratch[w * 2 + 1]);
    }
    *rec = make_double2(dphi, fphi);
  }
}

// End of step for a tile: psi_{k+1/2} from the incident fluxes the accepted
// iterate was computed from (src = the buffer the last iteration read) and
// psi_{k-1/2}; copies the accepted scalar flux to phi_res (and phi_out).
template <int CH>
__device__ inline void tile_end(const StepArgs &a, const TileDev &t, const double *src,
                                const double *psi_prev, double *psi_next, const double *phi_acc,
                                double *phi_out, double *lds) {
  const int N = a.N, K = 2 * N, P = K + 2, KS = (2 * K) / 4;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, W = blockDim.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const double *F = a.frag_ed + (size_t)t.region * a.frag_ed_stride + lane;
  const double *ce = a.c_ed + (size_t)t.region * a.c_ed_stride;
  double *ldp = lds + (kTileCells + 2) * P;
  double f0[CH];
  if (wave < a.Met) load_frags<CH>(f0, F + (size_t)wave * KS * 64, 0, KS);
  for (int i = threadIdx.x; i < t.nc * 4; i += blockDim.x) {
    const double v = phi_acc[(size_t)t.c0 * 4 + i];
    a.phi_res[(size_t)t.c0 * 4 + i] = v;
    if (phi_out) phi_out[(size_t)t.c0 * 4 + i] = v;
  }
  const RowBlock blk[2] = {neighbour_block(lds, src, t, K), own_block(ldp, psi_prev, t, K)};
  copy_blocks_to_lds(blk, 2, K, P);
  __syncthreads();
  reflect_ghosts(lds, P, t, N, a.J, a.bcl, a.bcr);
  auto aload = [&](int ks) {
    const int k = ks * 4 + kq;
    if (k < N) return lds[(col + 2) * P + k];
    if (k < K) return lds[col * P + k];
    return ldp[col * P + (k - K)];
  };
  for (int rt = wave; rt < a.Met; rt += W) {
    const d4 acc = mma_rowtile<CH>(F + (size_t)rt * KS * 64, KS, rt == wave, f0, aload);
    const int row = rt * 16 + col;
    if (row < K) {
      const double cv = ce[row];
      for (int i = 0; i < 4; ++i) {
        const int cl = kq + 4 * i;
        if (cl < t.nc) psi_next[(size_t)(t.c0 + cl) * K + row] = acc[i] + cv;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// Start of step `cur` of the current solve: gh for every tile, and the
// previous step's last iterate moved into buffer 0 when it sits in buffer 1
// (each work-group moves its own rows).  The first thread of work-group 0
// opens the step in the control block without touching the fields the other
// work-groups read here.  Does nothing while a queued solve is stalled.
template <int CH>
__global__ __launch_bounds__(256) void k_step_begin(StepArgs a) {
  extern __shared__ double lds[];
  const StepCtl c = *a.ctl;
  if (c.stalled) return;
  const int parity = c.psi_base ^ (c.cur & 1);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    StepCtl *ct = a.ctl;
    ct->total0 = c.total0 + c.fin_accepted;
    ct->status = kRunning;
    ct->step_parity = parity;
    ct->open = c.cur;
    ct->e_last = -1.0;
    ct->e_prev = -1.0;
  }
  const int ti = tile_of_block(blockIdx.x, a.ntiles);
  if (ti < 0) return;
  const TileDev t = a.tiles[ti];
  if (c.fin_accepted & 1) {
    const int K = 2 * a.N;
    const double2 *so = reinterpret_cast<const double2 *>(a.out1 + (size_t)(t.c0 + 1) * K);
    double2 *dout = reinterpret_cast<double2 *>(a.out0 + (size_t)(t.c0 + 1) * K);
    for (int i = threadIdx.x; i < t.nc * K / 2; i += blockDim.x) dout[i] = so[i];
    for (int i = threadIdx.x; i < t.nc * 4; i += blockDim.x)
      a.phi0[(size_t)t.c0 * 4 + i] = a.phi1[(size_t)t.c0 * 4 + i];
  }
  tile_begin<CH>(a, t, parity ? a.psi1 : a.psi0, lds);
}

// Iterate l = cb + node of the current step.  Every work-group first decides
// iterate l-1 from the residual records of the previous launch (and, for the
// strict rule, iterate l-2); a decided step ends the launch for everyone.
// All loads that do not depend on the decision are issued before it.
template <int CH>
__global__ __launch_bounds__(256) void k_oci_iterate(StepArgs a, int node, int cb) {
  extern __shared__ double lds[];
  __shared__ double red[2], red2[2], scratch[2 * kMaxWaves];
  const int l = cb + node;
  const int par = (l - 1) & 1;
  const double *src = par ? a.out1 : a.out0;
  double *dst = par ? a.out0 : a.out1;
  const double *phi_old = par ? a.phi1 : a.phi0;
  double *phi_new = par ? a.phi0 : a.phi1;
  const double2 *recs = reinterpret_cast<const double2 *>(a.partial);
  const size_t slot = (size_t)a.ntiles;
  RecRegs r1, r2;
  if (l >= 2) rec_issue(r1, recs + ((l - 1) % 3) * slot, a.ntiles);
  const bool strict_prev = a.strict && l - 2 >= 2;
  if (strict_prev) rec_issue(r2, recs + ((l - 2) % 3) * slot, a.ntiles);
  const int ti = tile_of_block(blockIdx.x, a.ntiles);
  if (ti < 0) return;
  const TileDev t = a.tiles[ti];
  const StepCtl c = *a.ctl;
  IterPrefetch<CH> pf;
  iterate_prefetch<CH>(pf, a, t, src, phi_old, lds);
  if (c.stalled || c.status != kRunning) return;
  if (l >= 2) {
    rec_finish(r1, recs + ((l - 1) % 3) * slot, a.ntiles, red, scratch);
    double e_before = -1.0;
    if (strict_prev) {
      rec_finish(r2, recs + ((l - 2) % 3) * slot, a.ntiles, red2, scratch);
      e_before = rel_change(red2[0], red2[1]);
    }
    double e;
    const int dn = stop_rule(l - 1, red[0], red[1], 0, e_before, 2, a.tol, a.strict, a.max_iters,
                             &e);
    if (dn != kRunning) {
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        StepCtl *ct = a.ctl;
        ct->accepted = l - 1;
        ct->e_last = e;
        ct->status = dn;
      }
      return;
    }
  }
  iterate_compute<CH>(pf, a, t, src, dst, phi_new, lds, scratch,
                      reinterpret_cast<double2 *>(a.partial) + (l % 3) * slot + ti);
}

// End of the open step, whose last launched iterate is `last`: decides that
// iterate if no launch has decided the step yet, then computes psi_{k+1/2}
// and copies the accepted scalar flux (also to phi_out[open] when phi_out is
// given).  A step that is still undecided (or went non-finite) stalls the
// queue instead: the host resumes it.  The step's record is written either
// way; a decided step advances the solve's step counter.
template <int CH>
__global__ __launch_bounds__(256) void k_step_end(StepArgs a, double *phi_out, int last) {
  extern __shared__ double lds[];
  __shared__ double red[2], red2[2], scratch[2 * kMaxWaves];
  const double2 *recs = reinterpret_cast<const double2 *>(a.partial);
  const size_t slot = (size_t)a.ntiles;
  RecRegs r1, r2;
  rec_issue(r1, recs + (last % 3) * slot, a.ntiles);
  const bool strict_prev = a.strict && last - 1 >= 2;
  if (strict_prev) rec_issue(r2, recs + ((last - 1) % 3) * slot, a.ntiles);
  const StepCtl c = *a.ctl;
  if (c.stalled) return;
  const bool leader = blockIdx.x == 0 && threadIdx.x == 0;
  const int step = c.open;
  int status = c.status, L = c.accepted;
  double e_last = c.e_last;
  if (status == kRunning) {
    rec_finish(r1, recs + (last % 3) * slot, a.ntiles, red, scratch);
    double e_before = -1.0;
    if (strict_prev) {
      rec_finish(r2, recs + ((last - 1) % 3) * slot, a.ntiles, red2, scratch);
      e_before = rel_change(red2[0], red2[1]);
    }
    status = stop_rule(last, red[0], red[1], 0, e_before, 2, a.tol, a.strict, a.max_iters,
                       &e_last);
    L = last;
  }
  const bool decided = status != kRunning && status != kNonFinite;
  // the outcome goes to fields no work-group of this launch reads
  if (leader) {
    StepCtl *ct = a.ctl;
    ct->fin_accepted = L;
    ct->fin_status = status;
    ct->fin_e = e_last;
    if (a.rec) {
      a.rec[step].accepted = L;
      a.rec[step].status = status;
      a.rec[step].e_last = e_last;
    }
    if (decided) ct->cur = step + 1;
    else ct->stalled = 1;
  }
  if (!decided) return;
  const int parity = c.step_parity;
  const double *src = ((L - 1) & 1) ? a.out1 : a.out0;   // read by iterate L
  const double *phi_acc = (L & 1) ? a.phi1 : a.phi0;     // written by iterate L
  const int ti = tile_of_block(blockIdx.x, a.ntiles);
  if (ti < 0) return;
  const TileDev t = a.tiles[ti];
  tile_end<CH>(a, t, src, parity ? a.psi1 : a.psi0, parity ? a.psi0 : a.psi1, phi_acc,
               phi_out ? phi_out + (size_t)step * a.J * 4 : nullptr, lds);
}

template __global__ void k_step_begin<4>(StepArgs);
template __global__ void k_step_begin<8>(StepArgs);
template __global__ void k_step_begin<16>(StepArgs);
template __global__ void k_oci_iterate<4>(StepArgs, int, int);
template __global__ void k_oci_iterate<8>(StepArgs, int, int);
template __global__ void k_oci_iterate<16>(StepArgs, int, int);
template __global__ void k_step_end<4>(StepArgs, double *, int);
template __global__ void k_step_end<8>(StepArgs, double *, int);
template __global__ void k_step_end<16>(StepArgs, double *, int);

}  // namespace ocik
