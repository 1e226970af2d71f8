// One-cell inversion hot path: per-step constant, the block-Jacobi iteration
// and the end of step (Sec. "One-Cell Inversion (OCI)").
//
// For every cell j of region r the iteration solves (A - S) Psi_j = c_j with
// the incident fluxes of c^+ / c^- taken from the neighbours' previous
// iterate.  c_j is linear in (incident fluxes, psi_{k-1/2}, Q), and the
// scattering block S couples the angles only through the cell's four scalar
// fluxes (rank 4), so an iteration is applied in structured form:
//
//   phi_j^(l+1)       = H_r inc_j^(l) + h_j        (4 rows of the reduced
//                                                  operator, FP64 MFMA)
//   out_{j,m}^(l+1)   = g'_{j,m} + (two rows of A_m^{-1}) (s_r phi_j^(l+1)
//                                  + |mu_m| inc_{j,m})   (per angle, VALU)
//   [g'; h]_j         = from psi_{k-1/2,j} and Q_r  (once per step)
//   psi_{k+1/2,j,m}   = from inc_j^(L-1), psi_{k-1/2,j} and phi_j^(L)
//                                                  (end of step, per angle)
//
// which is the same iteration as solving every cell's dense system with its
// LU factors, with the products associated differently: O(N) work per cell.
// A work-group owns a 16-cell tile of one region; the scalar-flux rows run on
// v_mfma_f64_16x16x4f64 with the tile's incident fluxes as the A operand (one
// cell per MFMA row, gathered from the neighbours' outgoing rows staged in
// LDS) and the operator rows, packed in fragment order and L2-resident, as B.
//
// Launches: k_oci_iterate (one iterate), k_oci_iterate2 (two) and
// k_oci_iterateK (three or four: halo cells recomputed level by level) each
// write their iterates and per-tile residual records; an extra work-group of
// every iteration launch reduces the previous launch's records into the
// per-iterate e.  No launch waits on a decision: k_step_end applies the
// stopping rule to the iterates of the batch, forms psi_{k+1/2} from the
// accepted one and the next step's constant, and (inside a replayed window)
// computes iterate 1 of the next step.  A step still undecided stalls the
// queue (a control-block flag every kernel checks) and the host resumes it.
// Mixed precision (k_oci_inner) iterates an FP32 correction between FP64
// iterates.
#include "oci_kernels.h"
#include "plan.h"

namespace ocik {

// A block of consecutive rows (row length K doubles, K even) copied from
// global memory into LDS rows of pitch P; LDS rows rows .. cap-1 are filled
// with copies (see copy_load).
struct RowBlock {
  const double *src;   // first row in global memory
  double *dst;         // first LDS row
  int rows;            // rows to copy
  int cap;             // LDS rows owned by the block (rows .. cap-1 hold copies)
};

// Staged copy: the first batch of every thread's elements (NB pairs of
// doubles) is held in registers between issue_copy (loads) and finish_copy
// (LDS stores and any further batches), so the loads can be issued early.
// A kernel built for one angle count sizes NB to stage its whole block in
// that one batch (copy_batch): each further batch is one more memory round
// trip before the tile's work can start.
constexpr int kCopyBatch = 4, kCopyMax = 9;
template <int NB>
struct CopyRegsN {
  double2 v[NB];
};
using CopyRegs = CopyRegsN<kCopyBatch>;

// Pairs per thread that stage `rows` rows of 2 NF doubles with the
// work-group of NF's step kernels (64 min(ceil(2 NF / 16), 4) threads) in
// one batch, within kCopyBatch .. kCopyMax; kCopyBatch for any N (NF = 0).
constexpr int copy_batch(int NF, int rows) {
  const int w = (2 * NF + 15) / 16 < 4 ? (2 * NF + 15) / 16 : 4;
  const int need = NF ? (rows * NF + 64 * w - 1) / (64 * w) : kCopyBatch;
  return need < kCopyBatch ? kCopyBatch : (need > kCopyMax ? kCopyMax : need);
}

__device__ __forceinline__ int copy_total(const RowBlock *blk, int nblk, int h, int *off1) {
  const int n0 = blk[0].cap * h;
  *off1 = n0;
  return nblk > 1 ? n0 + blk[1].cap * h : n0;
}

// Element i of the staged blocks.  Loads are unconditional, from a clamped
// valid address: LDS rows past a block's rows receive copies of its last
// element, which no kernel uses (they are the rows of cells past the tile,
// whose results are discarded).  So a thread's loads issue back to back with
// no branch and no use of the value before the LDS store.
__device__ __forceinline__ double2 copy_load(const RowBlock *blk, int nblk, int h, int off1,
                                             int i) {
  const bool second = nblk > 1 && i >= off1;
  const int li = second ? i - off1 : i;
  const double *src = second ? blk[1].src : blk[0].src;
  const int n = (second ? blk[1].rows : blk[0].rows) * h;
  return reinterpret_cast<const double2 *>(src)[min(li, n - 1)];
}

__device__ __forceinline__ void copy_store(const RowBlock *blk, int nblk, int h, int off1, int P,
                                           int i, double2 v) {
  const int b = (nblk > 1 && i >= off1) ? 1 : 0;
  const int li = b ? i - off1 : i;
  const int r = li / h, c2 = li - r * h;
  *reinterpret_cast<double2 *>(blk[b].dst + r * P + 2 * c2) = v;
}

template <int NB>
__device__ inline void issue_copy(CopyRegsN<NB> &cr, const RowBlock *blk, int nblk, int K) {
  const int h = K / 2;
  int off1;
  const int total = copy_total(blk, nblk, h, &off1);
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int i = threadIdx.x + q * blockDim.x;
    cr.v[q] = copy_load(blk, nblk, h, off1, min(i, total - 1));   // stored only if i < total
  }
}

template <int NB>
__device__ inline void finish_copy(const CopyRegsN<NB> &cr, const RowBlock *blk, int nblk, int K,
                                   int P) {
  const int h = K / 2;
  int off1;
  const int total = copy_total(blk, nblk, h, &off1);
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int i = threadIdx.x + q * blockDim.x;
    if (i < total) copy_store(blk, nblk, h, off1, P, i, cr.v[q]);
  }
  for (int base = threadIdx.x + NB * blockDim.x; base < total;
       base += kCopyBatch * blockDim.x) {
    double2 v[kCopyBatch];
#pragma unroll
    for (int q = 0; q < kCopyBatch; ++q) {
      const int i = base + q * blockDim.x;
      v[q] = copy_load(blk, nblk, h, off1, min(i, total - 1));
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
// (Fragments past KS are loads of the last valid one, never used: every MFMA
// loop skips k-steps past KS.)
__device__ __forceinline__ void load_frags(double (&f)[CH], const double *Fr, int base, int KS) {
#pragma unroll
  for (int i = 0; i < CH; ++i) f[i] = Fr[(size_t)min(base + i, KS - 1) * 64];
}

// The iteration operator G is packed k-major per lane group: lane group kq
// (lanes 16kq .. 16kq+15) holds k = kq*KS + ks in k-step ks, so a lane's A
// values for consecutive k-steps are consecutive in one LDS row.  With VEC
// (KS a multiple of 4; every k-step range starts at a multiple of 4) they are
// read four at a time as two 16-byte reads ahead of their MFMAs.
template <bool VEC>
__device__ __forceinline__ void a_quad(const double *p, int ks, int KS, double (&v)[4]) {
  if (ks < KS) {
    const double2 x = *reinterpret_cast<const double2 *>(p + ks);
    const double2 y = *reinterpret_cast<const double2 *>(p + ks + 2);
    v[0] = x.x;
    v[1] = x.y;
    v[2] = y.x;
    v[3] = y.y;
  }
}

// acc += A * B over k-steps kb .. min(kb+NP, ke)-1 with the fragments in f;
// p = this lane's A values (k-step ks at p[ks]).
template <int NP, bool VEC>
__device__ __forceinline__ void mma_quads(d4 &acc, const double (&f)[NP], int kb, int ke,
                                          const double *p, int KS) {
  if (VEC) {
#pragma unroll
    for (int g = 0; g < NP; g += 4) {
      double v[4] = {0.0, 0.0, 0.0, 0.0};
      a_quad<VEC>(p, kb + g, KS, v);
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (kb + g + i < ke) acc = mfma16x16x4(v[i], f[g + i], acc);
    }
  } else {
#pragma unroll
    for (int i = 0; i < NP; ++i)
      if (kb + i < ke) acc = mfma16x16x4(p[kb + i], f[i], acc);
  }
}

// One row tile of G over all KS k-steps; the first CH fragments may come
// preloaded.
template <int CH, bool VEC>
__device__ __forceinline__ d4 mma_rowtile_g(const double *Fr, int KS, bool first_loaded,
                                            const double (&f0)[CH], const double *p) {
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  int base = 0;
  if (first_loaded) {
    mma_quads<CH, VEC>(acc, f0, 0, KS, p, KS);
    base = CH;
  }
  for (; base < KS; base += CH) {
    double f[CH];
    load_frags<CH>(f, Fr, base, KS);
    mma_quads<CH, VEC>(acc, f, base, KS, p, KS);
  }
  return acc;
}

// ---------------------------------------------------------------------------
// Tile routines
// ---------------------------------------------------------------------------

// The tile of this work-group.  Tiles are listed in work-group order (the
// host assigns consecutive tiles to the work-groups of one XCD, which the
// hardware dispatches round-robin over the 8 XCDs, so a region's operator is
// read into few L2s and neighbouring tiles share an L2).  With ARGT the
// packed descriptors travel in the kernel arguments: the descriptor load
// issues with the other argument loads, and no data load waits on a table.
// (wg: the tile index of this work-group within its problem: blockIdx.x,
// or the entry of an ensemble launch's work queue)
template <bool ARGT>
__device__ __forceinline__ TileDev blk_desc(const StepArgs &a, int wg) {
  TileDev t;
  if (ARGT) {
    const uint32_t w = a.tile_word[wg];
    t.c0 = (int)(w & ((1u << kArgTileCellBits) - 1));
    t.nc = (int)((w >> kArgTileCellBits) & 15u) + 1;
    t.region = (int)(w >> 22);
    t.pad = 0;
  } else {
    t = a.tiles[wg];
  }
  return t;
}

// ring buffer of iterate l >= 1 of a step whose iterates use ring half `half`
__device__ __forceinline__ int ring_buf(const StepArgs &a, int l, int half) {
  return half * a.nbuf + l % a.nbuf;
}
__device__ __forceinline__ double *out_at(const StepArgs &a, int b) {
  return a.outb + (size_t)b * a.out_stride;
}
__device__ __forceinline__ double *phi_at(const StepArgs &a, int b) {
  return a.phib + (size_t)b * a.phi_stride;
}
// Residual-record slot of iterate l of a step of ring half `half` (one set of
// nbuf per half, so that an end of step that starts the next step's iterate
// 1 never overwrites records it still reads).
__device__ __forceinline__ size_t rec_slot(const StepArgs &a, int l, int half) {
  return (size_t)(half * a.nbuf + l % a.nbuf) * a.ntiles;
}

// ---------------------------------------------------------------------------
// The structured apply
// ---------------------------------------------------------------------------
// Cell j's solution of (A - S) psi = c satisfies A_m psi_m = c_m + s phi
// angle by angle, phi = W psi its scalar flux (4 values: the scattering
// coupling of the angles has rank 4).  An OCI iteration therefore needs the
// dense reduced operator only for the new scalar flux,
//   phi^(l+1) = H inc^(l) + h            (H: the 4 scalar-flux rows of G),
// and each outgoing pair of angle m then follows from two rows of A_m^{-1}:
//   out_{m,t} = g'_{m,t} + A_m^{-1}[o_t,:] (s phi^(l+1) + |mu| inc_m)
// with g'_{m,t} = A_m^{-1}[o_t,:] c_m(psi_{k-1/2}, Q) the step constant
// (o_t: the outgoing-corner rows at levels k and k+1/2).  This is the same
// iteration as [out; phi] = G inc + [g; h] with the products associated
// differently: O(N) work per cell for the outgoing fluxes instead of 4N^2.
// The per (region, angle) coefficients (kCoef doubles, built at setup):
//   [6t + c]  s A^{-1}[o_t][c], c = 0..3   [6t + 4]  |mu| A^{-1}[o_t][in_0]
//   [6t + 5]  |mu| A^{-1}[o_t][in_1]       [12 + 3t] (dx Q / 4) sum_c A^{-1}[o_t][c]
//   [13 + 3t] (dx / (2 v dt)) A^{-1}[o_t][0]   [14 + 3t] (dx / (2 v dt)) A^{-1}[o_t][1]
// (in_0, in_1: the entering-corner rows at levels k and k+1/2), and for the
// end of step, rows r = 2, 3 of A^{-1} (psi_{k+1/2} at L and R), u = r - 2:
//   [18 + 9u + c] s A^{-1}[r][c]   [22 + 9u] (dx/(2 v dt)) A^{-1}[r][0]
//   [23 + 9u] (dx/(2 v dt)) A^{-1}[r][1]   [24 + 9u] |mu| A^{-1}[r][in_0]
//   [25 + 9u] |mu| A^{-1}[r][in_1]   [26 + 9u] (dx Q / 4) sum_c A^{-1}[r][c]

constexpr int kStepWaves = 4;   // most waves of a step kernel's work-group (256 threads)
constexpr int kPhiPre = 4;   // scalar-flux operator fragments prefetched per wave
constexpr int kGPre = 2;     // cells whose step constants a thread prefetches

// The step constant values a thread of gh_compute formed for its first
// cells and (wave 0) its (cell, component) h, for an iteration that follows
// in the same work-group with the same thread mapping.
struct GhOut {
  double gq[kGPre][2];
  double hv;
};

// Angle and cells of this thread in the per-(cell, angle) loops: angle
// tid mod N, cells tid / N + j * cstep (threads past cstep * N idle).
struct PairMap {
  int m, cl0, cstep;
  bool active;
  __device__ __forceinline__ explicit PairMap(int N) {
    const int tid = threadIdx.x;
    cstep = (int)blockDim.x / N;
    m = tid % N;
    cl0 = tid / N;
    active = tid < cstep * N;
  }
};

// Coefficients 2 i2 and 2 i2 + 1 of (region r, angle m): the table holds
// pairs of coefficients, pair-major ([R][kCoef/2][N] double2), so a thread
// loads two per instruction and consecutive angles are consecutive.
__device__ __forceinline__ double2 coef_pair(const StepArgs &a, int N, int r, int m, int i2) {
  return reinterpret_cast<const double2 *>(a.coef)[((size_t)r * (kCoef / 2) + i2) * N + m];
}

// n consecutive coefficients (n even, i0 even) of (region r, angle m).
template <int n>
__device__ __forceinline__ void coef_load(const StepArgs &a, int N, int r, int m, int i0,
                                          double (&c)[n]) {
#pragma unroll
  for (int i = 0; i < n; i += 2) {
    const double2 v = coef_pair(a, N, r, m, (i0 + i) / 2);
    c[i] = v.x;
    c[i + 1] = v.y;
  }
}

// The scalar-flux rows 2N .. 2N+3 of G and P: their row tile and the first of
// them within it (2N is a multiple of 4, so all four share one row tile).
__device__ __forceinline__ void phi_tile(int N, int *rt, int *off) {
  const int K = 2 * N;
  *rt = K / 16;
  *off = K % 16;
}

// k-steps of a row tile handled by wave w when it is split over W waves
// (range starts at multiples of 4; equal shares when KS allows).
__device__ __forceinline__ void phi_ksplit(int KS, int W, int w, int *kb, int *ke) {
  if (KS % (4 * W) == 0) {
    *kb = w * (KS / W);
    *ke = *kb + KS / W;
  } else {
    *kb = ((w * KS) / W) & ~3;
    *ke = w + 1 == W ? KS : (((w + 1) * KS) / W) & ~3;
  }
}

// The step constant of a tile from its psi rows in LDS (pitch P, cell c in
// row c): h (rows 2N .. 2N+3 of gh) = the scalar-flux rows of P psi + p on
// MFMA, k-steps split over the waves (f0: this wave's first fragments) and
// summed in a fixed order; g' (rows 0 .. 2N-1) per (cell, angle).
template <int CH, bool VEC, int NF>
__device__ __forceinline__ void gh_compute(const StepArgs &a, const TileDev &t, const double *rows,
                                  const double (&f0)[CH], const double (&cg)[6], GhOut &go,
                                  bool want_go) {
  __shared__ double hp[kStepWaves * 64];
  const int N = NF ? NF : a.N, K = 2 * N, P = K + 2, KS = K / 4;
  const int Mt = NF ? (2 * NF + 4 + 15) / 16 : a.Mt;
  const int W = (int)(blockDim.x >> 6);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col = lane & 15, kq = lane >> 4;
  const int ghp = Mt * 16;
  int prt, poff, kb, ke;
  phi_tile(N, &prt, &poff);
  phi_ksplit(KS, W, wave, &kb, &ke);
  {
    const double *Fp = a.frag_pv + (size_t)t.region * a.frag_pv_stride + lane +
                       (size_t)prt * KS * 64;
    const double *ap = rows + col * P + kq * KS;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    mma_quads<CH, VEC>(acc, f0, kb, ke, ap, KS);
    for (int base = kb + CH; base < ke; base += CH) {
      double f[CH];
      load_frags<CH>(f, Fp, base, ke);
      mma_quads<CH, VEC>(acc, f, base, ke, ap, KS);
    }
    hp[wave * 64 + lane] = 0.0;
    if (col >= poff && col < poff + 4) {
#pragma unroll
      for (int i = 0; i < 4; ++i) hp[wave * 64 + (kq + 4 * i) * 4 + col - poff] = acc[i];
    }
  }
  const PairMap pm(N);
  if (pm.active) {
    const double c0 = cg[0], c1 = cg[1], c2 = cg[2], c3 = cg[3], c4 = cg[4], c5 = cg[5];
    int j = 0;
    for (int cl = pm.cl0; cl < t.nc; cl += pm.cstep, ++j) {
      const double pl = rows[cl * P + 2 * pm.m], pr = rows[cl * P + 2 * pm.m + 1];
      const double g0 = c0 + c1 * pl + c2 * pr, g1 = c3 + c4 * pl + c5 * pr;
      *reinterpret_cast<double2 *>(a.gh + (size_t)(t.c0 + cl) * ghp + 2 * pm.m) =
          make_double2(g0, g1);
      if (want_go) {   // (entry j by selects: a run-time index would put go in scratch)
#pragma unroll
        for (int i = 0; i < kGPre; ++i)
          if (i == j) {
            go.gq[i][0] = g0;
            go.gq[i][1] = g1;
          }
      }
    }
  }
  __syncthreads();
  if (wave == 0) {
    const int cl = lane >> 2, comp = lane & 3;
    double v = 0.0;
    for (int w = 0; w < W; ++w) v += hp[w * 64 + lane];
    v += a.c_pv[(size_t)t.region * a.c_pv_stride + K + comp];
    if (cl < t.nc) a.gh[(size_t)(t.c0 + cl) * ghp + K + comp] = v;
    if (want_go) go.hv = v;
  }
}

// Fragments of P's scalar-flux row tile per batch in the end of step: a
// wave's whole share (KS / W k-steps) when the angle count is fixed and the
// share is below CH, so that no registers hold other waves' k-steps.
template <int NF, int CH>
constexpr int gh_batch() {
  if (!NF) return CH;
  const int w = (2 * NF + 15) / 16 < 4 ? (2 * NF + 15) / 16 : 4;
  const int share = (NF / 2) / w;
  return share >= CH ? CH : (share >= 4 ? share : 4);
}

// The first fragments of this wave's share of P's scalar-flux row tile.
template <int CH, int NF>
__device__ __forceinline__ void gh_frags(const StepArgs &a, const TileDev &t, double (&f0)[CH]) {
  const int N = NF ? NF : a.N, KS = (2 * N) / 4;
  const int W = (int)(blockDim.x >> 6);
  const int lane = threadIdx.x & 63;
  int prt, poff, kb, ke;
  phi_tile(N, &prt, &poff);
  phi_ksplit(KS, W, threadIdx.x >> 6, &kb, &ke);
  const double *F = a.frag_pv + (size_t)t.region * a.frag_pv_stride + lane;
  load_frags<CH>(f0, F + ((size_t)prt * KS + kb) * 64, 0, ke - kb);
}

// gh of a tile from psi_{k-1/2} in global memory.
template <int CH, bool VEC, int NF>
__device__ inline void tile_begin(const StepArgs &a, const TileDev &t, const double *psi_prev,
                                  double *lds) {
  const int N = NF ? NF : a.N, K = 2 * N, P = K + 2;
  double f0[CH], cg[6];
  gh_frags<CH, NF>(a, t, f0);
  coef_load<6>(a, N, t.region, (int)threadIdx.x % N, 12, cg);   // (the thread's angle)
  const RowBlock blk[1] = {own_block(lds, psi_prev, t, K)};
  copy_blocks_to_lds(blk, 1, K, P);
  __syncthreads();
  GhOut unused;
  gh_compute<CH, VEC, NF>(a, t, lds, f0, cg, unused, false);
}

// One OCI iteration of a tile, in two phases: iterate_prefetch issues every
// load that does not need LDS (the first operator chunk of the wave's share
// of the scalar-flux row tile, this thread's out coefficients and step
// constants, the old scalar flux, and the neighbour rows, staged into LDS by
// iterate_compute).  iterate_compute runs the scalar-flux rows on MFMA with
// their k-steps split over the waves and summed in LDS in a fixed order;
// wave 0 forms the 64 (cell, component) scalar fluxes and the tile's
// residual record; then every thread forms its outgoing pairs.

template <int CH, int NF, int NB = copy_batch(NF, kTileCells + 2)>
struct IterPrefetch {
  double fp[kPhiPre];
  double cf[12];          // out coefficients of this thread's angle
  double gq[kGPre][2];    // g' of its first cells
  double hv, po;          // scalar-flux constant and previous value of this lane's (cell, component)
  CopyRegsN<NB> cr;       // the neighbour rows
};

// Problem shape seen by the iteration kernel: compile-time constants when the
// kernel is built for one angle count NF (> 0), else from the arguments.
template <int NF>
struct IterShape {
  int N, K, KS, Mto, Mt, W;
  __device__ __forceinline__ explicit IterShape(const StepArgs &a)
      : N(NF ? NF : a.N),
        K(2 * N),
        KS(K / 4),
        Mto(NF ? (2 * NF + 15) / 16 : a.Mto),
        Mt(NF ? (2 * NF + 4 + 15) / 16 : a.Mt),
        W(NF ? ((2 * NF + 15) / 16 < 4 ? (2 * NF + 15) / 16 : 4) : (int)(blockDim.x >> 6)) {}
};

// go: the step constants already in registers (the end of step that formed
// them, same work-group and thread mapping), else loaded.
template <int CH, int NF, int NB>
__device__ __forceinline__ void iterate_prefetch(IterPrefetch<CH, NF, NB> &pf, const StepArgs &a, const TileDev &t,
                                        const double *src, const double *phi_old, double *lds,
                                        const GhOut &go, bool have_go) {
  const IterShape<NF> sh(a);
  const int N = sh.N, K = sh.K, KS = sh.KS, W = sh.W;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const double *F = a.frag_it + (size_t)t.region * a.frag_it_stride + lane;
  const int ghp = sh.Mt * 16;
  int prt, poff, kb, ke;
  phi_tile(N, &prt, &poff);
  phi_ksplit(KS, W, wave, &kb, &ke);
  load_frags<kPhiPre>(pf.fp, F + ((size_t)prt * KS + kb) * 64, 0, ke - kb);
  const PairMap pm(N);
  coef_load<12>(a, N, t.region, pm.m, 0, pf.cf);
  if (have_go) {
#pragma unroll
    for (int j = 0; j < kGPre; ++j) {
      pf.gq[j][0] = go.gq[j][0];
      pf.gq[j][1] = go.gq[j][1];
    }
  } else {
#pragma unroll
    for (int j = 0; j < kGPre; ++j) {
      const int cl = min(pm.cl0 + j * pm.cstep, t.nc - 1);   // (used only for cells < nc)
      {   // (a pair, 16-byte aligned: 2m is even and rows are 16 doubles apart)
        const double2 g2 =
            *reinterpret_cast<const double2 *>(a.gh + (size_t)(t.c0 + cl) * ghp + 2 * pm.m);
        pf.gq[j][0] = g2.x;
        pf.gq[j][1] = g2.y;
      }
    }
  }
  const int cl = lane >> 2, comp = lane & 3;
  const int cc = t.c0 + min(cl, t.nc - 1);   // (used by wave 0 for cells < nc)
  pf.hv = have_go ? go.hv : a.gh[(size_t)cc * ghp + K + comp];
  pf.po = phi_old[(size_t)cc * 4 + comp];
  const RowBlock blk[1] = {neighbour_block(lds, src, t, K)};
  issue_copy(pf.cr, blk, 1, K);
}

// The outgoing pairs of iterate_compute for this thread's angle and cells.
template <int NF, int CH, int NB>
__device__ __forceinline__ void iterate_pairs(const IterPrefetch<CH, NF, NB> &pf, const StepArgs &a,
                                     const TileDev &t, double *dst, const double *lds,
                                     const double *phif, const PairMap &pm, int wm) {
  const int N = NF ? NF : a.N, K = 2 * N, P = K + 2;
  const int ghp = (NF ? (2 * NF + 4 + 15) / 16 : a.Mt) * 16;
  const int m = pm.m;
  const bool pos = 2 * m >= N;   // mu > 0: enters from the left neighbour (LDS row c)
  int j = 0;
  for (int cl = pm.cl0; cl < t.nc; cl += pm.cstep, ++j) {
    const double *in = lds + (pos ? cl : cl + 2) * P + 2 * m;
    const double *ph = phif + cl * 4;
    const double i0 = in[0], i1 = in[1];
    const double f0 = ph[0], f1 = ph[1], f2 = ph[2], f3 = ph[3];
    const size_t cell = (size_t)(t.c0 + cl);
    double g0, g1;
    if (j < kGPre) {
      g0 = pf.gq[j < kGPre ? j : 0][0];
      g1 = pf.gq[j < kGPre ? j : 0][1];
    } else {
      g0 = a.gh[cell * ghp + 2 * m];
      g1 = a.gh[cell * ghp + 2 * m + 1];
    }
    const double *c = pf.cf;
    const double o0 = g0 + c[0] * f0 + c[1] * f1 + c[2] * f2 + c[3] * f3 + c[4] * i0 + c[5] * i1;
    const double o1 = g1 + c[6] * f0 + c[7] * f1 + c[8] * f2 + c[9] * f3 + c[10] * i0 + c[11] * i1;
    if (wm & 1) *reinterpret_cast<double2 *>(dst + (cell + 1) * K + 2 * m) = make_double2(o0, o1);
    // the defect against the iterate this one was computed from (its own
    // row is staged in LDS row cl+1)
    if (wm & 2)
      *reinterpret_cast<float2 *>(a.dlt + (cell + 1) * K + 2 * m) =
          make_float2((float)(o0 - lds[(cl + 1) * P + 2 * m]),
                      (float)(o1 - lds[(cl + 1) * P + 2 * m + 1]));
  }
}

// Computes the tile's iterate; wave 0 writes its residual record (rec).
// Returns early (no stores) when `skip` is set (a stalled queue).  wm: bit 0
// stores the outgoing fluxes (always the scalar flux), bit 1 also the FP32
// defect against the iterate this one started from (mixed precision).
template <int CH, bool VEC, int NF, int NB>
__device__ __forceinline__ void iterate_compute(const IterPrefetch<CH, NF, NB> &pf, const StepArgs &a,
                                       const TileDev &t, const double *src, double *dst,
                                       double *phi_new, double *lds, double *phis, double *phif,
                                       double2 *rec, bool skip, int wm) {
  const IterShape<NF> sh(a);
  const int N = sh.N, K = sh.K, P = K + 2, KS = sh.KS, W = sh.W;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col = lane & 15, kq = lane >> 4;
  const double *F = a.frag_it + (size_t)t.region * a.frag_it_stride + lane;
  {
    const RowBlock blk[1] = {neighbour_block(lds, src, t, K)};
    finish_copy(pf.cr, blk, 1, K, P);
  }
  __syncthreads();
  if (skip) return;
  reflect_ghosts(lds, P, t, N, a.J, a.bcl, a.bcr);
  // incident flux of cell c, entry k: k < N from the right neighbour
  // (LDS row c+2), k >= N from the left neighbour (LDS row c).  With the
  // k-major packing k = kq*KS + ks, so k < N exactly for kq < 2.
  const double *ap = lds + (kq < 2 ? col + 2 : col) * P + kq * KS;
  int prt, poff, kb, ke;
  phi_tile(N, &prt, &poff);
  phi_ksplit(KS, W, wave, &kb, &ke);
  // this wave's partial scalar flux, [cell][component] in LDS (zero if none)
  double *my_phis = phis + wave * 64;
  my_phis[lane] = 0.0;
  {
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    const double *Fp = F + (size_t)prt * KS * 64;
    mma_quads<kPhiPre, VEC>(acc, pf.fp, kb, ke, ap, KS);
    for (int base = kb + kPhiPre; base < ke; base += CH) {
      double f[CH];
      load_frags<CH>(f, Fp, base, ke);
      mma_quads<CH, VEC>(acc, f, base, ke, ap, KS);
    }
    if (col >= poff && col < poff + 4) {
#pragma unroll
      for (int i = 0; i < 4; ++i) my_phis[(kq + 4 * i) * 4 + col - poff] = acc[i];
    }
  }
  __syncthreads();
  double dphi = 0.0, fphi = 0.0;   // wave 0: this lane's residual values
  if (wave == 0) {
    // scalar flux of (cell, component) = lane: the waves' partials in order
    const int cl = lane >> 2, comp = lane & 3;
    double s = 0.0;
    for (int w = 0; w < W; ++w) s += phis[w * 64 + lane];
    const double v = s + pf.hv;
    phif[lane] = v;
    if (cl < t.nc) {
      phi_new[(size_t)(t.c0 + cl) * 4 + comp] = v;
      if (wm & 2) a.dphi32[(size_t)(t.c0 + cl) * 4 + comp] = (float)(v - pf.po);
      dphi = isfinite(v) ? fabs(v - pf.po) : __builtin_nan("");
      fphi = fabs(v);
    }
  }
  __syncthreads();
  // outgoing pairs of this thread's angle for its cells; then wave 0 reduces
  // the residual record (after the pairs, so that no wave waits for it)
  const PairMap pm(N);
  if (pm.active) iterate_pairs<NF>(pf, a, t, dst, lds, phif, pm, wm);
  if (wave == 0) {
    dphi = wave_nan_max(dphi);
    fphi = wave_max(fphi);
    if (lane == 0) *rec = make_double2(dphi, fphi);
  }
}


// End of step for a tile.  The accepted iterate L solved every cell's
// system (A - S) psi = c with the incident fluxes of iterate L-1 (src = the
// buffer iterate L read) and gave its scalar flux phi_L = W psi.  With the
// scattering source s phi_L known, each angle's 4x4 block separates:
// A_m psi_m = c_m + s phi_L (Sec. "One-Cell Inversion (OCI)", the cell
// equations with the scattering term moved to the right-hand side), so
// psi_{k+1/2} (rows (k+1/2)L, (k+1/2)R of psi_m) is two rows of A_m^{-1} times
// a 4-vector per (cell, angle): O(N) per cell instead of a 2N x 4N product.
// Also copies the accepted scalar flux to phi_res (and phi_out), and forms
// the next step's gh from psi_{k+1/2} (kept in LDS).
// The loads of tile_end that depend on the accepted iterate or the step,
// all issued before its first store (a load issued after a store waits for
// it): the accepted scalar flux (one value per thread, nc * 4 <= 64 <=
// blockDim), this thread's angle's psi_{k-1/2} values, and the neighbour
// rows of the iterate the accepted one was computed from (src; into LDS
// later).
// (psi_{k-1/2} of a thread's first kGPre cells; at N = 64, four cells per
// thread, the other two (n2) once the staged rows have left their registers,
// so that the end of step fits 128 registers: four work-groups per CU)
template <int NF>
struct EndPre {
  static constexpr int n = kGPre, n2 = NF == 64 ? 2 : 0;
};
template <int NF>
struct EndLoads {
  double pq[EndPre<NF>::n][2], pv;
  CopyRegs cr;   // (one batch of kCopyBatch: the end of step has no registers to spare)
};

template <int NF>
__device__ __forceinline__ void end_loads(const StepArgs &a, const TileDev &t, const double *src,
                                          const double *psi_prev, const double *phi_acc,
                                          double *lds, EndLoads<NF> &el) {
  const int N = NF ? NF : a.N, K = 2 * N;
  const int pi = threadIdx.x;
  el.pv = pi < t.nc * 4 ? phi_acc[(size_t)t.c0 * 4 + pi] : 0.0;
  const PairMap pm(N);
#pragma unroll
  for (int j = 0; j < EndPre<NF>::n; ++j) {
    const int cl = min(pm.cl0 + j * pm.cstep, t.nc - 1);   // (used only for cells < nc)
    const double2 p2 =
        *reinterpret_cast<const double2 *>(psi_prev + (size_t)(t.c0 + cl) * K + 2 * pm.m);
    el.pq[j][0] = p2.x;
    el.pq[j][1] = p2.y;
  }
  const RowBlock blk[1] = {neighbour_block(lds, src, t, K)};
  issue_copy(el.cr, blk, 1, K);
}

// (el: the loads of end_loads for these arguments when `loaded`, else
// filled here)
template <int CH, bool VEC, int NF>
__device__ __forceinline__ void tile_end(const StepArgs &a, const TileDev &t, const double *src,
                                const double *psi_prev, double *psi_next, const double *phi_acc,
                                double *phi_out, double *lds, GhOut &go, bool want_go,
                                EndLoads<NF> &el, bool loaded) {
  constexpr int NQ = EndPre<NF>::n, CHG = gh_batch<NF, CH>();
  __shared__ double sphi[4 * kTileCells];
  double fg[CHG];   // P fragments for the next step's gh, issued early
  gh_frags<CHG, NF>(a, t, fg);
  const int N = NF ? NF : a.N, K = 2 * N, P = K + 2;
  double *ldn = lds + (kTileCells + 2) * P;   // psi_{k+1/2} of the tile's cells
  const PairMap pm(N);
  const int m = pm.m;
  const bool pos = 2 * m >= N;   // mu > 0: enters from the left neighbour (LDS row c)
  double e[18];   // this thread's angle's coefficients of psi_{k+1/2}
  coef_load<18>(a, N, t.region, m, 18, e);
  if (!loaded) end_loads<NF>(a, t, src, psi_prev, phi_acc, lds, el);
  const int pi = threadIdx.x;
  const double pv = el.pv;
  const double(&pq)[NQ][2] = el.pq;
  const RowBlock blk[1] = {neighbour_block(lds, src, t, K)};
  const auto &cr = el.cr;
  if (pi < t.nc * 4) {
    a.phi_res[(size_t)t.c0 * 4 + pi] = pv;
    if (phi_out) phi_out[(size_t)t.c0 * 4 + pi] = pv;
    sphi[pi] = pv;
  }
  finish_copy(cr, blk, 1, K, P);
  constexpr int NQ2 = EndPre<NF>::n2 > 0 ? EndPre<NF>::n2 : 1;
  double pq2[NQ2][2];   // (cells NQ .. NQ+n2-1 of the thread)
#pragma unroll
  for (int q = 0; q < EndPre<NF>::n2; ++q) {
    const int cl = min(pm.cl0 + (NQ + q) * pm.cstep, t.nc - 1);   // (used only for cells < nc)
    const double2 p2 =
        *reinterpret_cast<const double2 *>(psi_prev + (size_t)(t.c0 + cl) * K + 2 * m);
    pq2[q][0] = p2.x;
    pq2[q][1] = p2.y;
  }
  __syncthreads();
  reflect_ghosts(lds, P, t, N, a.J, a.bcl, a.bcr);
  if (pm.active) {
    int j = 0;
    for (int cl = pm.cl0; cl < t.nc; cl += pm.cstep, ++j) {
      const double *pp = psi_prev + (size_t)(t.c0 + cl) * K + 2 * m;
      const double *ph = sphi + cl * 4;
      const double *in = lds + (pos ? cl : cl + 2) * P + 2 * m;
      const double f0 = ph[0], f1 = ph[1], f2 = ph[2], f3 = ph[3];
      double pl, pr;
      if (j < NQ) {   // (entry j by selects: a run-time index would put pq in scratch)
        pl = pq[0][0];
        pr = pq[0][1];
#pragma unroll
        for (int q = 1; q < NQ; ++q)
          if (q == j) {
            pl = pq[q][0];
            pr = pq[q][1];
          }
      } else if (j < NQ + EndPre<NF>::n2) {
        pl = pq2[0][0];
        pr = pq2[0][1];
#pragma unroll
        for (int q = 1; q < EndPre<NF>::n2; ++q)
          if (NQ + q == j) {
            pl = pq2[q][0];
            pr = pq2[q][1];
          }
      } else {
        pl = pp[0];
        pr = pp[1];
      }
      const double i0 = in[0], i1 = in[1];
      const double x2 = e[8] + e[0] * f0 + e[1] * f1 + e[2] * f2 + e[3] * f3 + e[4] * pl +
                        e[5] * pr + e[6] * i0 + e[7] * i1;
      const double x3 = e[17] + e[9] * f0 + e[10] * f1 + e[11] * f2 + e[12] * f3 + e[13] * pl +
                        e[14] * pr + e[15] * i0 + e[16] * i1;
      *reinterpret_cast<double2 *>(psi_next + (size_t)(t.c0 + cl) * K + 2 * m) =
          make_double2(x2, x3);
      ldn[cl * P + 2 * m] = x2;
      ldn[cl * P + 2 * m + 1] = x3;
    }
  }
  // the next step's gh from psi_{k+1/2}, so that a queued step that
  // follows needs no step start (the g' coefficients loaded only now, when
  // the registers of the psi phase are free)
  double cg[6];
  coef_load<6>(a, N, t.region, m, 12, cg);
  __syncthreads();
  gh_compute<CHG, VEC, NF>(a, t, ldn, fg, cg, go, want_go);
}

// Start of step `cur` of the current solve: gh for every tile from
// psi_{k-1/2}.  Needed only where no end of step has computed it (the first
// step of a queue).  Does nothing while a queued solve is stalled.
template <int CH, bool ARGT, bool VEC, int NF>
__device__ __forceinline__ void step_begin_body(const StepArgs &a, int wg, double *lds) {
  const TileDev t = blk_desc<ARGT>(a, wg);   // (read with the control block)
  const StepCtl c = *a.ctl;
  if (c.stalled) return;
  const int parity = c.psi_base ^ (c.cur & 1);
  tile_begin<CH, VEC, NF>(a, t, parity ? a.psi1 : a.psi0, lds);
}

template <int CH, bool ARGT, bool VEC, int NF>
__global__ __launch_bounds__(256) void k_step_begin(StepArgs a) {
  extern __shared__ double lds[];
  step_begin_body<CH, ARGT, VEC, NF>(a, blockIdx.x, lds);
}

// Iterate l = cb + node of the open step: always computed (the step's
// decision is taken by the end-of-step kernel from the residual of every
// iterate).  Iterate 1 starts from the previous step's accepted iterate
// (buffer fin_buf) and opens the step: its first thread records the step
// index and that buffer for the end of step.  Work-group 0 also reduces the
// residual records iterate l-1 left and stores its e in dec, off the other
// work-groups' path.  Nothing is stored while a queued solve is stalled.
// The extra work-group of an iteration launch (block index ntiles): the e of
// iterates l - j*rstep, j = nred .. 1, from their residual records into dec,
// beside the tiles instead of on one tile's path.
// The step's first launch (l = 1, or 2 after a fused end of step) records
// the open step and the buffer of its iterate 0 for the end of step.  Stored
// last in the launch: on this GPU a load issued after a store waits for that
// store to complete.
__device__ __forceinline__ void open_step(const StepArgs &a, int l, int cur, int fb, int stalled,
                                          int wg) {
  if (l <= 2 && wg == 0 && threadIdx.x == 0 && !stalled) {
    a.ctl->open = cur;
    a.ctl->base_buf = fb;
  }
}

__device__ inline void reduce_prev(const StepArgs &a, int l, int rstep, int nred, int half,
                                   double *red, double *scratch) {
  const int stalled = a.ctl->stalled;
  const double2 *recs = reinterpret_cast<const double2 *>(a.partial);
  for (int j = nred; j >= 1; --j) {
    const int lp = l - j * rstep;
    if (lp < 1) continue;
    RecRegs r1;
    rec_issue(r1, recs + rec_slot(a, lp, half), a.ntiles);
    rec_finish(r1, recs + rec_slot(a, lp, half), a.ntiles, red, scratch);
    if (threadIdx.x == 0 && !stalled) a.dec[lp % a.nbuf] = rel_change(red[0], red[1]);
  }
}

// rmode: bits 0-1 the stride of the judged iterates (1; 2 for mixed
// precision, whose FP64 iterates also store their FP32 defect), bit 2 the
// outgoing fluxes are not stored (a mixed-precision iterate 1 that a
// correction follows: nothing reads them), bit 3 the defect is not stored
// (the last FP64 iterate a queued step planned; a resumed step forms it).
template <int CH, bool ARGT, bool VEC, int NF>
__device__ __forceinline__ void oci_iterate_body(const StepArgs &a, int wg, double *lds, int node,
                                                 int cb, int half, int rmode, int nred) {
  __shared__ double red[2], scratch[2 * kMaxWaves], phis[4 * 64], phif[64];
  const int rstep = rmode & 3;
  const int wm = ((rmode & 4) ? 0 : 1) | ((rstep == 2 && !(rmode & 8)) ? 2 : 0);
  const int l = cb + node;
  if (wg == a.ntiles) {
    reduce_prev(a, l, rstep, nred, half, red, scratch);
    return;
  }
  // iterate 0 of the step: the previous step's accepted iterate.  The step's
  // first launch (l = 1, or l = 2 when the previous end of step computed
  // iterate 1) opens it.
  int b0 = ring_buf(a, l - 1, half), cur = 0, fb = 0;
  if (l <= 2) {
    fb = a.ctl->fin_buf;
    cur = a.ctl->cur;
    if (l == 1) b0 = fb;
  }
  const double *src = out_at(a, b0);
  double *dst = out_at(a, ring_buf(a, l, half));
  const double *phi_old = phi_at(a, b0);
  double *phi_new = phi_at(a, ring_buf(a, l, half));
  const int ti = wg;   // the tile's residual record
  const TileDev t = blk_desc<ARGT>(a, wg);
  IterPrefetch<CH, NF> pf;
  const GhOut none{};
  iterate_prefetch<CH, NF>(pf, a, t, src, phi_old, lds, none, false);
  const int stalled = a.ctl->stalled;
  iterate_compute<CH, VEC, NF>(pf, a, t, src, dst, phi_new, lds, phis, phif,
                      reinterpret_cast<double2 *>(a.partial) + rec_slot(a, l, half) + ti,
                      stalled != 0, wm);
  open_step(a, l, cur, fb, stalled, wg);
}

template <int CH, bool ARGT, bool VEC, int NF>
__global__ __launch_bounds__(256, 3) void k_oci_iterate(StepArgs a, int node, int cb, int half,
                                                        int rmode, int nred) {
  extern __shared__ double lds[];
  oci_iterate_body<CH, ARGT, VEC, NF>(a, blockIdx.x, lds, node, cb, half, rmode, nred);
}

// The FP32 defect of FP64 iterate l of the open step (mixed precision)
// against the point it was computed from (iterate l-1, or the step's start
// for l = 1): outgoing part into correction buffer 0, scalar-flux part into
// dphi32.  For a resumed step whose last queued FP64 iterate did not store
// it.  Grid-stride over the cells' K outgoing values and 4 scalar fluxes.
__global__ __launch_bounds__(256) void k_defect(StepArgs a, int l, int half) {
  const int K = 2 * a.N;
  const int bp = l == 1 ? a.ctl->base_buf : ring_buf(a, l - 1, half);
  const int bl = ring_buf(a, l, half);
  const double *x = out_at(a, bl), *y = out_at(a, bp);
  const double *xp = phi_at(a, bl), *yp = phi_at(a, bp);
  const size_t n_out = (size_t)a.J * K, n_phi = (size_t)a.J * 4;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_out + n_phi;
       i += (size_t)gridDim.x * blockDim.x) {
    if (i < n_out) {
      const size_t e = K + i;   // (row 0 is the ghost row)
      a.dlt[e] = (float)(x[e] - y[e]);
    } else {
      const size_t e = i - n_out;
      a.dphi32[e] = (float)(xp[e] - yp[e]);
    }
  }
}

// ---------------------------------------------------------------------------
// Two iterates per launch
// ---------------------------------------------------------------------------
// Iterate l+1 of a tile needs iterate l of its own cells and of the cell on
// each side (its halo cells).  The launch stages iterate l-1 of the cells
// c0-2 .. c0+nc+1 (LDS block A, row r <-> cell c0-2+r), computes iterate l of
// its own cells as k_oci_iterate does and of the halo cells' entering halves
// (their scalar flux as four dot products on the vector units, with their
// own region's operator), keeps iterate l in LDS (block B, row r <-> cell
// c0-1+r) and computes iterate l+1 of its own cells from it.  Both iterates
// are stored with their residual records.  Every halo value is computed from
// the same inputs by the same arithmetic as by the tile that owns the cell,
// so the two copies agree to rounding order of the dot products.

// Left (pos = true) or right halo cell hc at iterate l: its scalar flux from
// its incident fluxes (entry k < N from the row of its right neighbour, k >= N
// from its left neighbour's), then its outgoing pairs in the angles entering
// the tile into `orow`.  One wave.
template <int NF>
__device__ inline void halo_iterate(const StepArgs &a, int hc, const double *left,
                                    const double *right, bool pos, double *orow) {
  const int N = NF ? NF : a.N, K = 2 * N;
  const int lane = threadIdx.x & 63;
  const int ghp = (NF ? (2 * NF + 4 + 15) / 16 : a.Mt) * 16;
  const int r = a.cell_region[hc];
  // row q of the wave (lanes 16q .. 16q+15) forms component q
  const int q = lane >> 4;
  const double *Fq = a.phig + ((size_t)r * 4 + q) * K;   // scalar-flux row q of G
  double acc = 0.0;
  for (int k = lane & 15; k < K; k += 16) {
    const double v = k < N ? right[k] : left[k];
    acc += Fq[k] * v;
  }
  acc = row_sum16(acc);
  const double *gh = a.gh + (size_t)hc * ghp;
  double ph[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) ph[c] = lane_f64(acc, 16 * c) + gh[K + c];
  for (int j = lane; j < N / 2; j += 64) {
    const int m = pos ? N / 2 + j : j;
    double cf[12];
    coef_load<12>(a, N, r, m, 0, cf);
    const double *in = (pos ? left : right) + 2 * m;   // the halo cell's entering flux
    const double i0 = in[0], i1 = in[1];
    orow[2 * m] = gh[2 * m] + cf[0] * ph[0] + cf[1] * ph[1] + cf[2] * ph[2] + cf[3] * ph[3] +
                  cf[4] * i0 + cf[5] * i1;
    orow[2 * m + 1] = gh[2 * m + 1] + cf[6] * ph[0] + cf[7] * ph[1] + cf[8] * ph[2] +
                      cf[9] * ph[3] + cf[10] * i0 + cf[11] * i1;
  }
}

// Reflecting edge: a ghost row takes the boundary cell's mirror-angle values
// (left ghost: entries N .. 2N-1, right ghost: 0 .. N-1).
__device__ __forceinline__ void mirror_row(double *ghost, const double *cell, int N, bool left) {
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const int e = left ? N + i : i;
    const int m = e >> 1, tl = e & 1;
    ghost[e] = cell[2 * (N - 1 - m) + tl];
  }
}

// The scalar-flux rows of one iterate of the tile's own cells from the rows
// at `base` (row 0 = cell c0-1): MFMA partials per wave into phis, summed by
// wave 0 with h into phif and stored to phi_out; the residual record's lane
// values against po (|change|, |value|) go to rv[0..63], rv[64..127] in LDS
// for flush_records.  Returns wave 0's value for its (cell, component).
template <int CH, bool VEC, int NF, int NP = kPhiPre>
__device__ inline double own_phi(const StepArgs &a, const TileDev &t, const double *base,
                                 const double (&fp)[NP], double hv, double po,
                                 double *phis, double *phif, double *phi_out, double *rv) {
  const IterShape<NF> sh(a);
  const int N = sh.N, K = sh.K, P = K + 2, KS = sh.KS, W = sh.W;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col = lane & 15, kq = lane >> 4;
  int prt, poff, kb, ke;
  phi_tile(N, &prt, &poff);
  phi_ksplit(KS, W, wave, &kb, &ke);
  double *my_phis = phis + wave * 64;
  my_phis[lane] = 0.0;
  {
    const double *Fp = a.frag_it + (size_t)t.region * a.frag_it_stride + lane +
                       (size_t)prt * KS * 64;
    const double *ap = base + (kq < 2 ? col + 2 : col) * P + kq * KS;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    mma_quads<NP, VEC>(acc, fp, kb, ke, ap, KS);
    for (int b = kb + NP; b < ke; b += CH) {
      double f[CH];
      load_frags<CH>(f, Fp, b, ke);
      mma_quads<CH, VEC>(acc, f, b, ke, ap, KS);
    }
    if (col >= poff && col < poff + 4) {
#pragma unroll
      for (int i = 0; i < 4; ++i) my_phis[(kq + 4 * i) * 4 + col - poff] = acc[i];
    }
  }
  __syncthreads();
  double v = 0.0;
  if (wave == 0) {
    const int cl = lane >> 2, comp = lane & 3;
    double s = 0.0;
    for (int w = 0; w < W; ++w) s += phis[w * 64 + lane];
    v = s + hv;
    phif[lane] = v;
    double dphi = 0.0, fphi = 0.0;
    if (cl < t.nc) {
      phi_out[(size_t)(t.c0 + cl) * 4 + comp] = v;
      dphi = isfinite(v) ? fabs(v - po) : __builtin_nan("");
      fphi = fabs(v);
    }
    rv[lane] = dphi;
    rv[64 + lane] = fphi;
  }
  __syncthreads();
  return v;
}

// The residual records of the launch's iterates l .. l+n-1 from their lane
// values (rv, 128 per iterate, after a barrier) into tile wg's slots: one
// wave per iterate, off the iterates' own path.
__device__ inline void flush_records(const StepArgs &a, int l, int n, int half, const double *rv,
                                     int wg) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, W = blockDim.x >> 6;
  for (int i = wave; i < n; i += W) {
    const double d = wave_nan_max(rv[i * 128 + lane]);
    const double f = wave_max(rv[i * 128 + 64 + lane]);
    if (lane == 0)
      reinterpret_cast<double2 *>(a.partial)[rec_slot(a, l + i, half) + wg] =
          make_double2(d, f);
  }
}

// Outgoing pairs of one iterate of the own cells (this thread's angle and
// cells) from the rows at `base` (row 0 = cell c0-1) and phif, to dst and,
// when given, to the LDS rows at `keep` (same layout as base).
template <int NF, int NG = kGPre>
__device__ inline void own_pairs(const StepArgs &a, const TileDev &t, const double *base,
                                 const double *phif, const double (&cf)[12],
                                 const double (&gq)[NG][2], double *dst, double *keep) {
  const int N = NF ? NF : a.N, K = 2 * N, P = K + 2;
  const int ghp = (NF ? (2 * NF + 4 + 15) / 16 : a.Mt) * 16;
  const PairMap pm(N);
  if (!pm.active) return;
  const int m = pm.m;
  const bool pos = 2 * m >= N;
  int j = 0;
  for (int cl = pm.cl0; cl < t.nc; cl += pm.cstep, ++j) {
    const double *in = base + (pos ? cl : cl + 2) * P + 2 * m;
    const double *ph = phif + cl * 4;
    const double i0 = in[0], i1 = in[1];
    const double f0 = ph[0], f1 = ph[1], f2 = ph[2], f3 = ph[3];
    const size_t cell = (size_t)(t.c0 + cl);
    double g0, g1;
    if (j < NG) {   // (entry j by selects: a run-time index would put gq in scratch)
      g0 = gq[0][0];
      g1 = gq[0][1];
#pragma unroll
      for (int i = 1; i < NG; ++i)
        if (i == j) {
          g0 = gq[i][0];
          g1 = gq[i][1];
        }
    } else {
      g0 = a.gh[cell * ghp + 2 * m];
      g1 = a.gh[cell * ghp + 2 * m + 1];
    }
    const double o0 = g0 + cf[0] * f0 + cf[1] * f1 + cf[2] * f2 + cf[3] * f3 + cf[4] * i0 +
                      cf[5] * i1;
    const double o1 = g1 + cf[6] * f0 + cf[7] * f1 + cf[8] * f2 + cf[9] * f3 + cf[10] * i0 +
                      cf[11] * i1;
    dst[(cell + 1) * K + 2 * m] = o0;
    dst[(cell + 1) * K + 2 * m + 1] = o1;
    if (keep) {
      keep[(cl + 1) * P + 2 * m] = o0;
      keep[(cl + 1) * P + 2 * m + 1] = o1;
    }
  }
}

template <int CH, bool ARGT, bool VEC, int NF>
__global__ __launch_bounds__(256, 2) void k_oci_iterate2(StepArgs a, int node, int cb, int half,
                                                         int nred) {
  extern __shared__ double lds[];
  __shared__ double red[2], scratch[2 * kMaxWaves], phis[4 * 64], phif[64], rv[2 * 128];
  const IterShape<NF> sh(a);
  const int N = sh.N, K = sh.K, P = K + 2, KS = sh.KS, W = sh.W;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l = cb + node;   // iterates l and l+1
  if (blockIdx.x == a.ntiles) {   // the e of the previous launch's iterates
    reduce_prev(a, l, 1, nred, half, red, scratch);
    return;
  }
  int b0 = ring_buf(a, l - 1, half), cur = 0, fb = 0;
  if (l <= 2) {   // the step's first launch opens it (as in k_oci_iterate)
    fb = a.ctl->fin_buf;
    cur = a.ctl->cur;
    if (l == 1) b0 = fb;
  }
  const double *src = out_at(a, b0);
  const double *phi_old = phi_at(a, b0);
  const int b1 = ring_buf(a, l, half), b2 = ring_buf(a, l + 1, half);
  const TileDev t = blk_desc<ARGT>(a, blockIdx.x);
  double *A = lds, *B = lds + kBlkA * P;
  const int ghp = sh.Mt * 16;
  // loads that need no LDS: the first operator chunk of this wave's share of
  // the scalar-flux row tile (the same for both iterates), this thread's out
  // coefficients and step constants, h and the old scalar flux, and the rows
  // of iterate l-1 (ghosted rows c0-1 .. c0+nc+2, clamped to the mesh)
  double fp[kPhiPre], cf[12], gq[kGPre][2];
  {
    int prt, poff, kb, ke;
    phi_tile(N, &prt, &poff);
    phi_ksplit(KS, W, wave, &kb, &ke);
    const double *F = a.frag_it + (size_t)t.region * a.frag_it_stride + lane;
    load_frags<kPhiPre>(fp, F + ((size_t)prt * KS + kb) * 64, 0, ke - kb);
  }
  const PairMap pm(N);
  {
    coef_load<12>(a, N, t.region, pm.m, 0, cf);
#pragma unroll
    for (int j = 0; j < kGPre; ++j) {
      const int cl = min(pm.cl0 + j * pm.cstep, t.nc - 1);
      {   // (a pair, 16-byte aligned: 2m is even and rows are 16 doubles apart)
        const double2 g2 =
            *reinterpret_cast<const double2 *>(a.gh + (size_t)(t.c0 + cl) * ghp + 2 * pm.m);
        gq[j][0] = g2.x;
        gq[j][1] = g2.y;
      }
    }
  }
  double hv, po;
  {
    const int cl = lane >> 2, comp = lane & 3;
    const int cc = t.c0 + min(cl, t.nc - 1);
    hv = a.gh[(size_t)cc * ghp + K + comp];
    po = phi_old[(size_t)cc * 4 + comp];
  }
  const int g_lo = max(t.c0 - 1, 0), g_hi = min(t.c0 + t.nc + 2, a.J + 1);
  const int r_lo = g_lo - t.c0 + 1;   // block A row of ghosted row g_lo
  const RowBlock blk[1] = {RowBlock{src + (size_t)g_lo * K, A + r_lo * P, g_hi - g_lo + 1,
                                    kBlkA - r_lo}};
  CopyRegs cr;
  issue_copy(cr, blk, 1, K);
  const int stalled = a.ctl->stalled;
  finish_copy(cr, blk, 1, K, P);
  __syncthreads();
  if (stalled) return;
  const bool hl = t.c0 > 0, hr = t.c0 + t.nc < a.J;   // halo cells (else ghost rows)
  // reflecting edges next to a halo cell: its outer ghost mirrors it
  if (hl && t.c0 == 1 && a.bcl == kBcReflect) mirror_row(A, A + P, N, true);
  if (hr && t.c0 + t.nc == a.J - 1 && a.bcr == kBcReflect)
    mirror_row(A + (t.nc + 3) * P, A + (t.nc + 2) * P, N, false);
  // reflecting edges of the tile itself (rows c0-1 .. c0+nc from A + P)
  reflect_ghosts(A + P, P, t, N, a.J, a.bcl, a.bcr);
  // iterate l: halo cells (one wave each), own cells
  const int wl = W - 1, wr = W >= 2 ? W - 2 : W - 1;
  if (hl && wave == wl) halo_iterate<NF>(a, t.c0 - 1, A, A + 2 * P, true, B);
  if (hr && wave == wr)
    halo_iterate<NF>(a, t.c0 + t.nc, A + (t.nc + 1) * P, A + (t.nc + 3) * P, false,
                     B + (t.nc + 1) * P);
  const double vl = own_phi<CH, VEC, NF>(a, t, A + P, fp, hv, po, phis, phif, phi_at(a, b1), rv);
  own_pairs<NF>(a, t, A + P, phif, cf, gq, out_at(a, b1), B);
  __syncthreads();
  // iterate l at the mesh edges: ghost rows of B
  if (!hl || !hr) {
    if (!hl) {
      if (a.bcl == kBcReflect) mirror_row(B, B + P, N, true);
      else for (int i = N + threadIdx.x; i < K; i += blockDim.x) B[i] = A[P + i];
    }
    if (!hr) {
      if (a.bcr == kBcReflect) mirror_row(B + (t.nc + 1) * P, B + t.nc * P, N, false);
      else for (int i = threadIdx.x; i < N; i += blockDim.x)
        B[(t.nc + 1) * P + i] = A[(t.nc + 2) * P + i];
    }
    __syncthreads();
  }
  // iterate l+1 of the own cells from B
  own_phi<CH, VEC, NF>(a, t, B, fp, hv, vl, phis, phif, phi_at(a, b2), rv + 128);
  own_pairs<NF>(a, t, B, phif, cf, gq, out_at(a, b2), nullptr);
  flush_records(a, l, 2, half, rv, blockIdx.x);
  open_step(a, l, cur, fb, stalled, blockIdx.x);
}

// ---------------------------------------------------------------------------
// KI iterates per launch (KI = 3, 4)
// ---------------------------------------------------------------------------
// The two-iterate scheme with a wider halo: the launch stages iterate l-1 of
// the cells c0-KI .. c0+nc+KI-1 and computes level after level, each level
// one cell narrower on each side (the own cells with MFMA, the halo cells on
// the vector units with their own region's operator, whole outgoing rows),
// alternating between two LDS blocks (row r <-> cell c0-KI+r).  Ghost rows of
// the mesh edges are re-formed at every level.  Every level's own iterate is
// stored with its residual record.
//
// What the halo cells need besides the rows is staged in LDS with the rows,
// so that no level waits on memory: the scalar-flux rows of G and the pair
// coefficients of the tile's region and of the regions before and after it
// (HF [3][4][K], k-major; HC [3][12][N], angle-major; region slot 0 before,
// 1 the tile's, 2 after), and each halo cell's step constants (HG
// [2(KI-1)][K+4]: halo slot i < KI-1 is cell c0-1-i, slot KI-1+i cell
// c0+nc+i) and region slot.  The host uses this kernel only when no region
// is narrower than KI-1 cells, so every halo cell is in one of the three.
// No level reads global memory: on this GPU a load issued after stores waits
// for those stores to complete.

//
// From N = 64 on ("lean" staging) the three regions' tables would not leave
// room for two work-groups per CU, so only the tile's own scalar-flux rows of
// G are staged (HF [4][K]) and no coefficients (HC empty): every thread keeps
// the coefficients of its angle in the tile's region in registers (a halo
// pair's angle is the thread's own angle, since the work-group's thread count
// is a multiple of N), and a halo cell in another region -- only tiles at a
// region boundary have one -- reads its region's rows and coefficients from
// memory.  Each thread also keeps the step constants of all its own cells and
// each wave all its operator fragments in registers, so that the levels of
// tiles inside a region read no global memory.
template <int NF, int KI>
struct HaloLds {
  static constexpr int K = 2 * NF;
  static constexpr int W = (2 * NF + 15) / 16 < 4 ? (2 * NF + 15) / 16 : 4;
  static constexpr int threads = 64 * W;
  static constexpr bool lean = NF >= 64;
  static constexpr int nF = (lean ? 4 : 12) * K, nC = lean ? 0 : 36 * NF;
  static constexpr int nG = 2 * (KI - 1) * (K + 4);
  static constexpr int total = nF + nC + nG;
  // staged in pairs of doubles (every segment has even length and offset)
  static constexpr int per_thread = (total / 2 + threads - 1) / threads;
  // step constants per thread (its cells) and operator fragments per wave
  static constexpr int NG = lean ? kTileCells * NF / threads : kGPre;
  static constexpr int NP = lean ? (K / 4) / W : kPhiPre;
  static_assert(!lean || threads % NF == 0, "a halo pair's angle is the thread's angle");
  static_assert(!lean || (K / 4) % (4 * W) == 0, "equal k-step shares per wave");
};

// Scalar flux of a halo cell from its neighbours' rows (left: cell c-1,
// right: c+1) at the level before: h + (scalar-flux rows of G) x incident,
// with the rows of G (hf, [4][K]) and the cell's step constants (hg) in LDS.
// One wave; the lanes of row q (16q .. 16q+15) return component q.
template <int NF>
__device__ inline double cell_phi(const double *left, const double *right, const double *hf,
                                  const double *hg) {
  constexpr int N = NF, K = 2 * N;
  const int lane = threadIdx.x & 63, q = lane >> 4;   // row q of the wave: component q
  double acc = 0.0;
  static_assert(K % 16 == 0, "a row of 16 lanes covers K in whole passes");
#pragma unroll
  for (int i = 0; i < K / 16; ++i) {
    const int k = (lane & 15) + 16 * i;
    const double v = k < N ? right[k] : left[k];
    acc += hf[q * K + k] * v;
  }
  return row_sum16(acc) + hg[K + q];
}

// Iterates l .. l+kk-1 (kk <= KI) of tile wg: the halo reaches kk-1 cells
// on each side at the first level, one fewer at each level after.  The LDS
// layout is that of KI levels whatever kk is.
template <int CH, bool ARGT, bool VEC, int NF, int KI>
__device__ __forceinline__ void oci_iterateK_body(const StepArgs &a, int wg, int node, int cb,
                                                  int half, int nred, int kk) {
  static_assert(NF > 0, "fixed angle count");
  using HL = HaloLds<NF, KI>;
  constexpr int RB = kTileCells + 2 * KI;   // rows per LDS block
  constexpr int NS = 2 * (KI - 1);          // halo slots
  extern __shared__ double lds[];
  __shared__ double red[2], scratch[2 * kMaxWaves], phis[4 * 64], phif[64], hph[NS][4],
      rv[KI * 128];
  __shared__ int hsel[NS];
  const IterShape<NF> sh(a);
  const int N = sh.N, K = sh.K, P = K + 2, KS = sh.KS, W = sh.W;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int l = cb + node;   // iterates l .. l+kk-1
  if (wg == a.ntiles) {   // the e of the previous launch's iterates
    reduce_prev(a, l, 1, nred, half, red, scratch);
    return;
  }
  const TileDev t = blk_desc<ARGT>(a, wg);
  // the staged regions: before, the tile's, after (clamped to the mesh)
  const int rg0 = max(t.region - 1, 0), rg2 = min(t.region + 1, a.R - 1);
  // (a select, not an indexed array: an array indexed at run time lives in
  // scratch memory)
  auto rg = [&](int rsl) { return rsl == 0 ? rg0 : (rsl == 1 ? t.region : rg2); };
  auto slot_cell = [&](int sl) { return sl < KI - 1 ? t.c0 - 1 - sl : t.c0 + t.nc + sl - (KI - 1); };
  int my_sel = 1;   // this thread's halo slot (threads < NS): its region slot
  if ((int)threadIdx.x < NS) {
    const int c = slot_cell(threadIdx.x);
    if (c >= 0 && c < a.J && a.cell_region[c] != t.region) my_sel = (int)threadIdx.x < KI - 1 ? 0 : 2;
  }
  int b0 = ring_buf(a, l - 1, half), cur = 0, fb = 0;
  if (l <= 2) {   // the step's first launch opens it (as in k_oci_iterate)
    fb = a.ctl->fin_buf;
    cur = a.ctl->cur;
    if (l == 1) b0 = fb;
  }
  const double *src = out_at(a, b0);
  const double *phi_old = phi_at(a, b0);
  double *X = lds, *Y = lds + RB * P;
  double *HF = lds + 2 * RB * P, *HC = HF + HL::nF, *HG = HC + HL::nC;
  const int cbase = t.c0 - KI;   // cell of LDS row 0
  auto row = [&](double *blk, int c) { return blk + (c - cbase) * P; };
  const int ghp = sh.Mt * 16;
  constexpr bool LEAN = HL::lean;
  constexpr int NG = HL::NG, NP = HL::NP;
  double fp[NP], cf[12], gq[NG][2];   // (fp, and cf unless lean: from the staged data, below)
  const PairMap pm(N);
  if (LEAN) coef_load<12>(a, N, t.region, pm.m, 0, cf);
  {
#pragma unroll
    for (int j = 0; j < NG; ++j) {
      const int cl = min(pm.cl0 + j * pm.cstep, t.nc - 1);
      {   // (a pair, 16-byte aligned: 2m is even and rows are 16 doubles apart)
        const double2 g2 =
            *reinterpret_cast<const double2 *>(a.gh + (size_t)(t.c0 + cl) * ghp + 2 * pm.m);
        gq[j][0] = g2.x;
        gq[j][1] = g2.y;
      }
    }
  }
  double hv, po;
  {
    const int cl = lane >> 2, comp = lane & 3;
    const int cc = t.c0 + min(cl, t.nc - 1);
    hv = a.gh[(size_t)cc * ghp + K + comp];
    po = phi_old[(size_t)cc * 4 + comp];
  }
  // iterate l-1 of cells c0-KI .. c0+nc+KI-1: ghosted rows c0-KI+1 .. c0+nc+KI,
  // clamped to the mesh and its two ghost rows
  const int g_lo = max(t.c0 - KI + 1, 0), g_hi = min(t.c0 + t.nc + KI, a.J + 1);
  const int r_lo = g_lo - 1 - cbase;
  const RowBlock blk[1] = {RowBlock{src + (size_t)g_lo * K, X + r_lo * P, g_hi - g_lo + 1,
                                    RB - r_lo}};
  CopyRegsN<copy_batch(NF, RB)> cr;
  issue_copy(cr, blk, 1, K);
  // the halo staging loads (HF, HC, HG in that order), two doubles at a time:
  // every segment (a region's 4 rows of G, its 12 coefficient rows, a halo
  // cell's step constants) is contiguous in memory with an even length
  double2 hreg[HL::per_thread];
#pragma unroll
  for (int i = 0; i < HL::per_thread; ++i) {
    const int idx = 2 * ((int)threadIdx.x + i * HL::threads);
    double2 v = make_double2(0.0, 0.0);
    const double *g = nullptr;
    if (idx < HL::nF) {
      const int rsl = LEAN ? 1 : idx / (4 * K), qk = LEAN ? idx : idx - rsl * 4 * K;
      g = a.phig + (size_t)rg(rsl) * 4 * K + qk;
    } else if (idx < HL::nF + HL::nC) {
      const int j = idx - HL::nF, rsl = j / (12 * N), cm = j - rsl * 12 * N;
      g = a.coef + (size_t)rg(rsl) * kCoef * N + cm;   // coefficients 0..11, all angles
    } else if (idx < HL::total) {
      const int j = idx - HL::nF - HL::nC, sl = j / (K + 4), e = j - sl * (K + 4);
      const int c = slot_cell(sl);
      if (c >= 0 && c < a.J) g = a.gh + (size_t)c * ghp + e;
    }
    if (g) v = *reinterpret_cast<const double2 *>(g);
    hreg[i] = v;
  }
  const int stalled = a.ctl->stalled;
  finish_copy(cr, blk, 1, K, P);
#pragma unroll
  for (int i = 0; i < HL::per_thread; ++i) {
    const int idx = 2 * ((int)threadIdx.x + i * HL::threads);
    if (idx < HL::total) *reinterpret_cast<double2 *>(HF + idx) = hreg[i];
  }
  if ((int)threadIdx.x < NS) hsel[threadIdx.x] = my_sel;
  __syncthreads();
  if (stalled) return;
  if (!LEAN) {
#pragma unroll
    for (int i = 0; i < 6; ++i) {   // region slot 1: the tile's
      const double2 v = reinterpret_cast<const double2 *>(HC + 12 * N)[i * N + pm.m];
      cf[2 * i] = v.x;
      cf[2 * i + 1] = v.y;
    }
  }
  {   // this wave's MFMA fragments of the scalar-flux rows of G (the k-major
      // packing of its row tile: lane 16 kq + r holds row r, k = kq KS + ks;
      // rows past the four scalar-flux rows are zero), from the staged rows
    int prt, poff, kb, ke;
    phi_tile(N, &prt, &poff);
    phi_ksplit(KS, W, wave, &kb, &ke);
    const int r = (lane & 15) - poff, kq = lane >> 4;
    const double *hf1 = HF + (LEAN ? 0 : 4 * K);   // the tile's region
#pragma unroll
    for (int q = 0; q < NP; ++q)
      fp[q] = (r >= 0 && r < 4) ? hf1[r * K + kq * KS + min(kb + q, KS - 1)] : 0.0;
  }
  const bool gl = cbase <= -1, gr = t.c0 + t.nc + KI - 1 >= a.J;   // ghost rows in the block
  if (gl && a.bcl == kBcReflect) mirror_row(row(X, -1), row(X, 0), N, true);
  if (gr && a.bcr == kBcReflect) mirror_row(row(X, a.J), row(X, a.J - 1), N, false);
  __syncthreads();
  double pl = po;   // wave 0: the previous level's scalar flux of its (cell, component)
  for (int s = 1; s <= kk; ++s) {
    const int lvl = l + s - 1;
    double *in = (s & 1) ? X : Y;
    double *out = (s & 1) ? Y : X;
    const int reach = kk - s;   // halo cells computed at this level on each side
    const int lo = max(t.c0 - reach, 0), hi = min(t.c0 + t.nc - 1 + reach, a.J - 1);
    const int nl = t.c0 - lo, nh = nl + hi - (t.c0 + t.nc - 1);
    // halo scalar fluxes, one wave per cell (the last waves first)
    for (int h = W - 1 - wave; h < nh; h += W) {
      const bool left = h < nl;
      const int c = left ? lo + h : t.c0 + t.nc + (h - nl);
      const int sl = left ? t.c0 - 1 - c : KI - 1 + c - (t.c0 + t.nc);
      const int hs = hsel[sl];
      const double *hf = LEAN ? (hs == 1 ? HF : a.phig + (size_t)rg(hs) * 4 * K)
                              : HF + hs * 4 * K;
      const double ph = cell_phi<NF>(row(in, c - 1), row(in, c + 1), hf, HG + sl * (K + 4));
      if ((lane & 15) == 0) hph[h][lane >> 4] = ph;
    }
    const int bl = ring_buf(a, lvl, half);
    pl = own_phi<CH, VEC, NF, NP>(a, t, row(in, t.c0 - 1), fp, hv, pl, phis, phif,
                                  phi_at(a, bl), rv + (s - 1) * 128);
    own_pairs<NF, NG>(a, t, row(in, t.c0 - 1), phif, cf, gq, out_at(a, bl),
                      s < kk ? row(out, t.c0 - 1) : nullptr);
    if (s == kk) {
      flush_records(a, l, kk, half, rv, wg);
      open_step(a, l, cur, fb, stalled, wg);
      break;
    }
    // the halo cells' outgoing rows (every angle: they feed the next level)
    for (int p = threadIdx.x; p < nh * N; p += blockDim.x) {
      const int h = p / N, m = p - h * N;
      const bool left = h < nl;
      const int c = left ? lo + h : t.c0 + t.nc + (h - nl);
      const int sl = left ? t.c0 - 1 - c : KI - 1 + c - (t.c0 + t.nc);
      double cc[12];   // pairs of coefficients, pair-major
      const int hs = hsel[sl];
      if (LEAN) {   // (m is this thread's angle: its own region's are in cf)
        if (hs == 1) {
#pragma unroll
          for (int i = 0; i < 12; ++i) cc[i] = cf[i];
        } else {
          coef_load<12>(a, N, rg(hs), m, 0, cc);
        }
      } else {
        const double2 *hc = reinterpret_cast<const double2 *>(HC + hs * 12 * N);
#pragma unroll
        for (int i = 0; i < 6; ++i) {
          const double2 v = hc[i * N + m];
          cc[2 * i] = v.x;
          cc[2 * i + 1] = v.y;
        }
      }
      const double *in2 = (2 * m >= N ? row(in, c - 1) : row(in, c + 1)) + 2 * m;
      const double i0 = in2[0], i1 = in2[1];
      const double *ph = hph[h];
      const double *g = HG + sl * (K + 4) + 2 * m;
      double *o = row(out, c) + 2 * m;
      o[0] = g[0] + cc[0] * ph[0] + cc[1] * ph[1] + cc[2] * ph[2] + cc[3] * ph[3] +
             cc[4] * i0 + cc[5] * i1;
      o[1] = g[1] + cc[6] * ph[0] + cc[7] * ph[1] + cc[8] * ph[2] + cc[9] * ph[3] +
             cc[10] * i0 + cc[11] * i1;
    }
    __syncthreads();
    // mesh edges at this level: ghost rows next to a boundary cell computed
    // here (a fixed ghost row is carried over from the level before, which
    // also computed that boundary cell)
    const bool el = gl && lo == 0, er = gr && hi == a.J - 1;
    if (el || er) {
      if (el) {
        if (a.bcl == kBcReflect) mirror_row(row(out, -1), row(out, 0), N, true);
        else for (int i = N + threadIdx.x; i < K; i += blockDim.x) row(out, -1)[i] = row(in, -1)[i];
      }
      if (er) {
        if (a.bcr == kBcReflect) mirror_row(row(out, a.J), row(out, a.J - 1), N, false);
        else for (int i = threadIdx.x; i < N; i += blockDim.x) row(out, a.J)[i] = row(in, a.J)[i];
      }
      __syncthreads();
    }
  }
}

template <int CH, bool ARGT, bool VEC, int NF, int KI>
__global__ __launch_bounds__(256, 2) void k_oci_iterateK(StepArgs a, int node, int cb, int half,
                                                         int nred) {
  oci_iterateK_body<CH, ARGT, VEC, NF, KI>(a, blockIdx.x, node, cb, half, nred, KI);
}

// The e of iterate l from its residual records into dec (one work-group),
// for problems with many tiles, where every work-group of the end of step
// reducing all records would cost ntiles^2 loads.
__device__ __forceinline__ void reduce_rec_body(const StepArgs &a, int l, int n, int half) {
  __shared__ double red[2], scratch[2 * kMaxWaves];
  const int stalled = a.ctl->stalled;
  for (int j = l - n + 1; j <= l; ++j) {   // iterates l-n+1 .. l
    const double2 *recs = reinterpret_cast<const double2 *>(a.partial) + rec_slot(a, j, half);
    RecRegs r1;
    rec_issue(r1, recs, a.ntiles);
    rec_finish(r1, recs, a.ntiles, red, scratch);
    if (threadIdx.x == 0 && !stalled) a.dec[j % a.nbuf] = rel_change(red[0], red[1]);
  }
}

// One work-group per iterate l-n+1 .. l (grid n): each reduces its own
// iterate's records and writes its own dec slot.
__global__ __launch_bounds__(256) void k_reduce_rec(StepArgs a, int l, int n, int half) {
  reduce_rec_body(a, l - n + 1 + (int)blockIdx.x, 1, half);
}

// End of the open step after iterates first .. last of it were launched
// (iterates before `first` were already found undecided): the first of them
// the stopping rule accepts (or stops at) is the step's iterate L.  The e of
// iterates before `last` come from dec, the e of `last` from its records.
// Then psi_{k+1/2} from the incident fluxes iterate L was computed from and
// psi_{k-1/2}, and the accepted scalar flux to phi_res (and phi_out[open]
// when given).  A step still undecided (or not finite) stalls the queue
// instead: the host resumes it.  The step's record is written either way; a
// decided step advances the solve's step counter.
// FUSE: built with the next step's first iterate (mode bit 16 selects it at
// run time); without it the kernel needs fewer registers.
// Work-groups per CU the end of step is built for (the register limit that
// follows: 128 for four, 168 for three): four at N = 64, whose 38.6 KiB of
// LDS per work-group also let four share a CU's 160 KiB; three otherwise.
template <int NF>
constexpr int kEndBlocks = NF == 64 ? 4 : 3;

template <int CH, bool ARGT, bool VEC, int NF, bool FUSE>
__device__ __forceinline__ void step_end_body(const StepArgs &a, int wg, double *lds,
                                              double *phi_out, int first, int last, int half,
                                              int rstep, int mode) {
  const bool pre = mode & 1, fuse = FUSE && ((mode >> 4) & 1);
  const int ntrail = (mode >> 1) & 7;   // iterates last-ntrail+1 .. last
  // (the tile's descriptor is read with the control block below, not after
  // it: the end loads wait for both)
  const TileDev t = blk_desc<ARGT>(a, wg);
  const double2 *recs = reinterpret_cast<const double2 *>(a.partial);
  RecRegs r1;
  if (!pre) rec_issue(r1, recs + rec_slot(a, last, half), a.ntiles);
  // the e of the earlier iterates (written by earlier launches), loaded with
  // the records, before the control block (at most kMaxRing + 1 <= 2 * 64 of them)
  __shared__ double sdec[kMaxRing + 1];
  const int l0 = first - 1 >= 1 ? first - 1 : first;
  const int nd = last - l0 + 1;
  const int i0 = threadIdx.x, i1 = threadIdx.x + blockDim.x;
  const double dv0 = i0 < nd ? a.dec[(l0 + i0) % a.nbuf] : 0.0;
  const double dv1 = i1 < nd ? a.dec[(l0 + i1) % a.nbuf] : 0.0;
  const StepCtl c = *a.ctl;
  if (c.stalled) return;
  if (i0 < nd) sdec[i0] = dv0;
  if (i1 < nd) sdec[i1] = dv1;
  __syncthreads();
  // the end usually accepts the last iterate: the loads of its end of step
  // are issued once the records are in, so that the reductions and the
  // decision hide their latency, and used if it is accepted
  const int parity = c.psi_base ^ (c.open & 1);
  const double *psi_prev = parity ? a.psi1 : a.psi0;
  const bool spec = last >= 2;
  EndLoads<NF> sel;
  if (pre && spec)
    end_loads<NF>(a, t, out_at(a, ring_buf(a, last - 1, half)), psi_prev,
                  phi_at(a, ring_buf(a, last, half)), lds, sel);
  // the e of the trailing iterates (those of the last launch) into sdec:
  // reduced by k_reduce_rec (many tiles: one reduction, not one per
  // work-group) or here, all of them in one pass over their records
  if (!pre) {
    double d[kMaxTrail], f[kMaxTrail];
#pragma unroll
    for (int j = 0; j < kMaxTrail; ++j) d[j] = f[j] = 0.0;
#pragma unroll
    for (int q = 0; q < kRecBatch; ++q) {
      d[0] = nan_max(d[0], r1.v[q].x);
      f[0] = nan_max(f[0], r1.v[q].y);
    }
    const double2 *rl = recs + rec_slot(a, last, half);
    for (int i = threadIdx.x + kRecBatch * blockDim.x; i < a.ntiles; i += blockDim.x) {
      d[0] = nan_max(d[0], rl[i].x);
      f[0] = nan_max(f[0], rl[i].y);
    }
    const double2 *rj[kMaxTrail];
#pragma unroll
    for (int j = 1; j < kMaxTrail; ++j) rj[j] = recs + rec_slot(a, j < ntrail ? last - j : last, half);
    for (int i = threadIdx.x; i < a.ntiles; i += blockDim.x) {
      double2 v[kMaxTrail];
#pragma unroll
      for (int j = 1; j < kMaxTrail; ++j) v[j] = j < ntrail ? rj[j][i] : make_double2(0.0, 0.0);
#pragma unroll
      for (int j = 1; j < kMaxTrail; ++j) {
        d[j] = nan_max(d[j], v[j].x);
        f[j] = nan_max(f[j], v[j].y);
      }
    }
    if (spec)
      end_loads<NF>(a, t, out_at(a, ring_buf(a, last - 1, half)), psi_prev,
                    phi_at(a, ring_buf(a, last, half)), lds, sel);
    // within each 16-lane row (DPP), then over the rows of all waves in LDS
    __shared__ double tscr[4 * kStepWaves][2 * kMaxTrail];
#pragma unroll
    for (int j = 0; j < kMaxTrail; ++j) {
      d[j] = row_reduce16(d[j], [](double x, double y) { return nan_max(x, y); });
      f[j] = row_reduce16(f[j], [](double x, double y) { return nan_max(x, y); });
    }
    if ((threadIdx.x & 15) == 0) {
#pragma unroll
      for (int j = 0; j < kMaxTrail; ++j) {
        tscr[threadIdx.x >> 4][2 * j] = d[j];
        tscr[threadIdx.x >> 4][2 * j + 1] = f[j];
      }
    }
    __syncthreads();
    if (threadIdx.x < ntrail) {
      const int j = threadIdx.x;
      double dd = 0.0, ff = 0.0;
      for (int r = 0; r < (int)(blockDim.x >> 4); ++r) {
        dd = nan_max(dd, tscr[r][2 * j]);
        ff = nan_max(ff, tscr[r][2 * j + 1]);
      }
      sdec[last - j - l0] = rel_change(dd, ff);
    }
    __syncthreads();
  }
  auto e_of = [&](int l) { return sdec[l - l0]; };
  const int step = c.open;
  // the first of the candidate iterates first, first + rstep, .. last that
  // the stopping rule stops at: every candidate judged by a thread of its
  // own (with the e of the candidate before it), the first one by an LDS min
  const int ncand = (last - first) / rstep + 1;
  // (the lambdas capture locals only: a reference to the argument block
  // captured by a closure would put a copy of it in scratch memory)
  const int strict = a.strict;
  auto e_before_of = [&](int i, int l) {
    if (i == 0) return (strict && first - 1 >= 2) ? e_of(first - 1) : -1.0;
    return l - rstep >= 2 ? e_of(l - rstep) : -1.0;
  };
  __shared__ int s_first;
  if (threadIdx.x == 0) s_first = ncand;
  __syncthreads();
  for (int i = threadIdx.x; i < ncand; i += blockDim.x) {
    const int l = first + i * rstep;
    if (stop_rule_e(l, e_of(l), e_before_of(i, l), 2, a.tol, a.strict, a.max_iters) != kRunning)
      atomicMin(&s_first, i);
  }
  __syncthreads();
  int status = kRunning, L = last;
  double e_acc = -1.0, e_pacc = -1.0;
  if (s_first < ncand) {
    L = first + s_first * rstep;
    status = stop_rule_e(L, e_of(L), e_before_of(s_first, L), 2, a.tol, a.strict, a.max_iters);
    e_acc = L >= 2 ? e_of(L) : -1.0;
    // (the iterate before it, for the a-posteriori bound the host reports)
    e_pacc = (L - rstep >= 2 && L - rstep >= l0) ? e_of(L - rstep) : -1.0;
  }
  const bool decided = status != kRunning && status != kNonFinite;
  // the outcome goes to fields no work-group of this launch reads (stored
  // after the work-group's loads: a load issued after a store waits for it)
  StepCtl *const ct = a.ctl;
  StepRecord *const rec = a.rec;
  double *const dec = a.dec;
  const int nbuf = a.nbuf, fin_buf = ring_buf(a, L, half);
  auto record = [&]() {
    if (wg == 0 && threadIdx.x == 0) {
      ct->fin_accepted = L;
      ct->fin_status = status;
      ct->fin_e = e_acc;
      ct->fin_e_prev = e_pacc;
      if (rec) {
        rec[step].accepted = L;
        rec[step].status = status;
        rec[step].e_last = e_acc;
        rec[step].e_prev = e_pacc;
      }
      if (decided) {
        ct->fin_buf = fin_buf;
        ct->cur = step + 1;
      } else {
        ct->stalled = 1;
        for (int i = 0; i < ntrail; ++i)   // for the resumed end
          dec[(last - i) % nbuf] = sdec[last - i - l0];
      }
    }
  };
  if (!decided) {
    record();
    return;
  }
  // iterate L was computed from iterate L-1 (iterate 0: the step's start)
  const double *src = out_at(a, L == 1 ? c.base_buf : ring_buf(a, L - 1, half));
  GhOut go;
  tile_end<CH, VEC, NF>(a, t, src, parity ? a.psi1 : a.psi0, parity ? a.psi0 : a.psi1,
                        phi_at(a, ring_buf(a, L, half)),
                        phi_out ? phi_out + (size_t)step * a.J * 4 : nullptr, lds,
                        go, fuse, sel, spec && L == last);
  if (!fuse) {
    record();
    return;
  }
  if constexpr (FUSE) {
    // iterate 1 of the next step (ring half half^1) from the accepted
    // iterate: every input is this tile's (its step constant, just formed) or
    // already in memory (the neighbours' accepted outgoing fluxes), so one
    // launch fewer
    __shared__ double phis[4 * 64], phif[64];
    __syncthreads();
    const int bl = ring_buf(a, L, half), bn = ring_buf(a, 1, half ^ 1);
    IterPrefetch<CH, NF, kCopyBatch> pf;   // (the end of step has no registers to spare)
    iterate_prefetch<CH, NF>(pf, a, t, out_at(a, bl), phi_at(a, bl), lds, go, true);
    // (mixed precision: iterate 1 is an FP64 iterate with its defect)
    iterate_compute<CH, VEC, NF>(pf, a, t, out_at(a, bl), out_at(a, bn), phi_at(a, bn), lds,
                                 phis, phif,
                                 reinterpret_cast<double2 *>(a.partial) +
                                     rec_slot(a, 1, half ^ 1) + wg,
                                 false, ((mode & 32) ? 0 : 1) | (rstep == 2 ? 2 : 0));
    record();
  }
}

template <int CH, bool ARGT, bool VEC, int NF>
__global__ __launch_bounds__(256, kEndBlocks<NF>) void k_step_end(StepArgs a, double *phi_out, int first,
                                                  int last, int half, int rstep, int mode) {
  extern __shared__ double lds[];
  step_end_body<CH, ARGT, VEC, NF, true>(a, blockIdx.x, lds, phi_out, first, last, half, rstep,
                                         mode);
}

// The end of step without the fused iterate (mode bit 16 ignored).
template <int CH, bool ARGT, bool VEC, int NF>
__global__ __launch_bounds__(256, kEndBlocks<NF>) void k_step_end_nf(StepArgs a, double *phi_out, int first,
                                                     int last, int half, int rstep, int mode) {
  extern __shared__ double lds[];
  step_end_body<CH, ARGT, VEC, NF, false>(a, blockIdx.x, lds, phi_out, first, last, half, rstep,
                                          mode);
}


// ---------------------------------------------------------------------------
// Mixed precision: FP64 defect correction with FP32 inner iterations
// ---------------------------------------------------------------------------
// The step's FP64 iterates y_o -> x'_o = T(y_o) (k_oci_iterate with rstep 2)
// also give the defect d_o = x'_o - y_o (outgoing and scalar-flux parts) in
// FP32.  The correction delta solves delta = G delta + d_o (the same
// block-Jacobi map without its constant part); the inner iterations run it
// from delta_1 = d_o in FP32 on MFMA, and the last of them forms the next FP64
// iterate y_{o+1} = y_o + delta.  Its FP64 iterate T(y_{o+1}) is then judged
// by the same stopping rule as plain OCI, so every accepted iterate is an FP64
// application of the operator.

typedef float f4 __attribute__((ext_vector_type(4)));

// Inner iteration i of the current correction over a tile, in the structured
// form of the FP64 iteration without its constant part:
//   e = H inc(delta_i)                 (the 4 scalar-flux rows of G, FP32 MFMA)
//   delta_{i+1}[phi]   = d[phi] + e
//   delta_{i+1}[out_m] = d[out_m] + (s A_m^{-1} rows) e + (|mu| A_m^{-1} rows) inc_m(delta_i)
// (the same coefficients as the FP64 iteration, in FP32), so an inner
// iteration moves 4 (6N + 8) bytes per cell.  delta_1 = d is buffer 0 of the
// correction buffers; the iterates alternate between buffers 1 and 2.  With
// ly > 0 (the last inner iteration) the FP64 iterate ly = (iterate ly-2, or
// the step's start for ly = 2) + delta_{i+1} is written to ring buffer ly
// instead of delta.  opens: the step's first launch (its iterate 1 came with
// the previous end of step), which opens the step.  Lane l of
// v_mfma_f32_16x16x4f32 holds rows 4 (l/16) ..
// 4 (l/16) + 3 of column l%16 of the product: four consecutive cells of one
// operator row.
constexpr int kDPre = 4;   // cells per thread whose defect is loaded up front
template <bool ARGT>
__global__ __launch_bounds__(256) void k_oci_inner(StepArgs a, int i, int ly, int half,
                                                   int opens) {
  constexpr int kFr = 8;   // operator k-steps of the wave's share loaded up front
  extern __shared__ double lds_raw[];
  float *lf = reinterpret_cast<float *>(lds_raw);
  __shared__ float phis32[kMaxWaves * 64], ef[64];
  const int N = a.N, K = 2 * N, KS = K / 4, P = K + 4, K4 = K / 4;
  const int W = (int)(blockDim.x >> 6);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col = lane & 15, kq = lane >> 4;
  const TileDev t = blk_desc<ARGT>(a, blockIdx.x);
  const float *src = a.dlt + (size_t)(i == 1 ? 0 : ((i & 1) ? 2 : 1)) * a.dlt_stride;
  float *dst = a.dlt + (size_t)((i & 1) ? 1 : 2) * a.dlt_stride;
  const float *dd = a.dlt;   // the defect d
  int prt, poff, kb, ke;
  phi_tile(N, &prt, &poff);
  phi_ksplit(KS, W, wave, &kb, &ke);
  const float *F = a.frag_it32 + (size_t)t.region * a.frag_it_stride + lane + (size_t)prt * KS * 64;
  const double *yb = nullptr, *ybp = nullptr;
  double *yo = nullptr, *yop = nullptr;
  // (the step's start is the previous step's accepted iterate, fin_buf until
  // this step's end: base_buf may be written by this very launch)
  int cur = 0, fb = 0;
  if (opens || ly == 2) {
    cur = a.ctl->cur;
    fb = a.ctl->fin_buf;
  }
  if (ly) {
    const int bb = ly == 2 ? fb : ring_buf(a, ly - 2, half);
    const int bo = ring_buf(a, ly, half);
    yb = out_at(a, bb);
    ybp = phi_at(a, bb);
    yo = out_at(a, bo);
    yop = phi_at(a, bo);
  }
  // loads that need no LDS first: this wave's first operator fragments, this
  // thread's coefficients, the defect (and with ly the FP64 point) of its
  // first cells, and wave 0's scalar-flux defect
  float f0[kFr];
#pragma unroll
  for (int q = 0; q < kFr; ++q) f0[q] = F[(size_t)min(kb + q, KS - 1) * 64];
  const PairMap pm(N);
  float cf[12];
  {
    double c[12];
    coef_load<12>(a, N, t.region, pm.m, 0, c);
#pragma unroll
    for (int q = 0; q < 12; ++q) cf[q] = (float)c[q];
  }
  float dq[kDPre][2];
  double yq[kDPre][2];
#pragma unroll
  for (int j = 0; j < kDPre; ++j) {
    const size_t cell = (size_t)(t.c0 + min(pm.cl0 + j * pm.cstep, t.nc - 1));
    const float2 v = *reinterpret_cast<const float2 *>(dd + (cell + 1) * K + 2 * pm.m);
    dq[j][0] = v.x;
    dq[j][1] = v.y;
    yq[j][0] = yq[j][1] = 0.0;
    if (ly) {
      const double2 y = *reinterpret_cast<const double2 *>(yb + (cell + 1) * K + 2 * pm.m);
      yq[j][0] = y.x;
      yq[j][1] = y.y;
    }
  }
  float dphi = 0.f;
  double yphi = 0.0;
  if (wave == 0) {
    const size_t ce = (size_t)(t.c0 + min(lane >> 2, t.nc - 1)) * 4 + (lane & 3);
    dphi = a.dphi32[ce];
    if (ly) yphi = ybp[ce];
  }
  const int stalled = a.ctl->stalled;
  {
    // rows of cells c0-1 .. c0+nc (ghosted rows c0 .. c0+nc+1) into LDS rows 0 .. nc+1
    const f4 *s4 = reinterpret_cast<const f4 *>(src + (size_t)t.c0 * K);
    const int n4 = (t.nc + 2) * K4;
    for (int e = threadIdx.x; e < n4; e += blockDim.x) {
      const int r = e / K4, k4 = e - r * K4;
      *reinterpret_cast<f4 *>(lf + r * P + 4 * k4) = s4[e];
    }
  }
  __syncthreads();
  if (stalled) return;
  // reflecting edges: the correction obeys the same (homogeneous) mirror map
  const bool rl = t.c0 == 0 && a.bcl == kBcReflect;
  const bool rr = t.c0 + t.nc == a.J && a.bcr == kBcReflect;
  if (rl)
    for (int e = N + threadIdx.x; e < K; e += blockDim.x) {
      const int m = e >> 1, tl = e & 1;
      lf[e] = lf[P + 2 * (N - 1 - m) + tl];
    }
  if (rr) {
    const int rg = t.nc + 1;
    for (int e = threadIdx.x; e < N; e += blockDim.x) {
      const int m = e >> 1, tl = e & 1;
      lf[rg * P + e] = lf[(rg - 1) * P + 2 * (N - 1 - m) + tl];
    }
  }
  if (rl || rr) __syncthreads();
  // this wave's share of e = H inc(delta): incident entry k of cell c from the
  // right neighbour (LDS row c+2) for k < N, from the left (row c) else
  {
    const float *ap = lf + (kq < 2 ? col + 2 : col) * P + kq * KS;
    f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < kFr; ++q)
      if (kb + q < ke) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ap[kb + q], f0[q], acc, 0, 0, 0);
    for (int ks = kb + kFr; ks < ke; ++ks)
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ap[ks], F[(size_t)ks * 64], acc, 0, 0, 0);
    if (col >= poff && col < poff + 4) {
#pragma unroll
      for (int r = 0; r < 4; ++r) phis32[wave * 64 + (4 * kq + r) * 4 + col - poff] = acc[r];
    }
  }
  __syncthreads();
  if (wave == 0) {   // e of (cell, component) = lane: the waves' partials in order
    float e = 0.f;
    for (int w = 0; w < W; ++w) e += phis32[w * 64 + lane];
    ef[lane] = e;
    const int cl = lane >> 2;
    if (ly && cl < t.nc) {
      const size_t ce = (size_t)(t.c0 + cl) * 4 + (lane & 3);
      yop[ce] = yphi + (double)(dphi + e);
    }
  }
  __syncthreads();
  const int m = pm.m;
  const bool pos = 2 * m >= N;
  int j = 0;
  for (int cl = pm.active ? pm.cl0 : t.nc; cl < t.nc; cl += pm.cstep, ++j) {
    const float *in = lf + (pos ? cl : cl + 2) * P + 2 * m;
    const float *e4 = ef + cl * 4;
    const float i0 = in[0], i1 = in[1];
    const float e0 = e4[0], e1 = e4[1], e2 = e4[2], e3 = e4[3];
    const size_t cell = (size_t)(t.c0 + cl);
    float d0, d1;
    double y0 = 0.0, y1 = 0.0;
    if (j < kDPre) {   // (entry j by selects: a run-time index would put dq in scratch)
      d0 = dq[0][0];
      d1 = dq[0][1];
      y0 = yq[0][0];
      y1 = yq[0][1];
#pragma unroll
      for (int q = 1; q < kDPre; ++q)
        if (q == j) {
          d0 = dq[q][0];
          d1 = dq[q][1];
          y0 = yq[q][0];
          y1 = yq[q][1];
        }
    } else {
      d0 = dd[(cell + 1) * K + 2 * m];
      d1 = dd[(cell + 1) * K + 2 * m + 1];
      if (ly) {
        y0 = yb[(cell + 1) * K + 2 * m];
        y1 = yb[(cell + 1) * K + 2 * m + 1];
      }
    }
    const float o0 = d0 + cf[0] * e0 + cf[1] * e1 + cf[2] * e2 + cf[3] * e3 + cf[4] * i0 +
                     cf[5] * i1;
    const float o1 = d1 + cf[6] * e0 + cf[7] * e1 + cf[8] * e2 + cf[9] * e3 + cf[10] * i0 +
                     cf[11] * i1;
    if (ly) {
      *reinterpret_cast<double2 *>(yo + (cell + 1) * K + 2 * m) =
          make_double2(y0 + (double)o0, y1 + (double)o1);
    } else {
      *reinterpret_cast<float2 *>(dst + (cell + 1) * K + 2 * m) = make_float2(o0, o1);
    }
  }
  if (opens) open_step(a, 1, cur, fb, stalled, blockIdx.x);
}

// Reflecting edge of a correction row in LDS (FP32): the ghost takes the
// boundary cell's mirror-angle values (left ghost: entries N .. 2N-1, right
// ghost: 0 .. N-1).
__device__ __forceinline__ void mirror_row32(float *ghost, const float *cell, int N, bool left) {
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const int e = left ? N + i : i;
    const int m = e >> 1, tl = e & 1;
    ghost[e] = cell[2 * (N - 1 - m) + tl];
  }
}

// e = H inc of the tile's cells from correction rows at `base` (row 1 + c holds
// own cell c; rows c and c + 2 its neighbours), on FP32 MFMA with the k-steps
// split over the waves; wave 0 sums the partials in order into ef[cell * 4 +
// component].  Ends with a barrier.
__device__ __forceinline__ void inner_phi(const float *base, int P, int KS, int kb, int ke,
                                          const float *F, const float (&f0)[8], float *phis32,
                                          float *ef) {
  constexpr int kFr = 8;
  const int W = (int)(blockDim.x >> 6);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col = lane & 15, kq = lane >> 4;
  int prt, poff;
  phi_tile(2 * KS, &prt, &poff);   // (2 KS = N: K = 2N columns, KS = K / 4)
  const float *ap = base + (kq < 2 ? col + 2 : col) * P + kq * KS;
  f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int q = 0; q < kFr; ++q)
    if (kb + q < ke) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ap[kb + q], f0[q], acc, 0, 0, 0);
  for (int ks = kb + kFr; ks < ke; ++ks)
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ap[ks], F[(size_t)ks * 64], acc, 0, 0, 0);
  if (col >= poff && col < poff + 4) {
#pragma unroll
    for (int r = 0; r < 4; ++r) phis32[wave * 64 + (4 * kq + r) * 4 + col - poff] = acc[r];
  }
  __syncthreads();
  if (wave == 0) {
    float e = 0.f;
    for (int w = 0; w < W; ++w) e += phis32[w * 64 + lane];
    ef[lane] = e;
  }
  __syncthreads();
}

// Two inner iterations per launch: delta_{i+1} of the tile's cells and of one
// halo cell on each side, kept in LDS, then delta_{i+2} of the tile's cells
// from it (delta_{i+1} never reaches memory).  A halo cell's scalar-flux
// correction is four dot products of its own region's rows of H with its
// incident corrections (FP64 sums of the FP32 values, one wave per halo
// cell), and only its pairs entering the tile are formed; every other value
// is formed as in k_oci_inner.  n: this launch's index within the correction
// (the buffers alternate per launch as in k_oci_inner); ly > 0: the
// correction's last launch, which forms FP64 iterate ly; opens as in
// k_oci_inner.  LDS: block A, the rows of delta_i of cells c0-2 .. c0+nc+1
// (row r <-> cell c0-2+r), and block B, delta_{i+1} of cells c0-1 .. c0+nc
// (row r <-> cell c0-1+r), pitch K+4 floats; then per halo side (0 left, 1
// right) the tables of its halo cell, loaded with the rows so that the halo
// work reads no global memory: HF [2][4][K] its region's rows of H, HC
// [2][12][N/2] the pair coefficients of its entering angles (entering angle
// j: N/2 + j on the left, j on the right), HD [2][N] its defect in those
// angles.  N <= 128 (the per-thread load slots below).
template <bool ARGT>
__global__ __launch_bounds__(256) void k_oci_inner2(StepArgs a, int n, int ly, int half,
                                                    int opens) {
  constexpr int kFr = 8;
  extern __shared__ double lds_raw[];
  __shared__ float phis32[kMaxWaves * 64], ef[64];
  const int N = a.N, K = 2 * N, KS = K / 4, P = K + 4, K4 = K / 4;
  float *A = reinterpret_cast<float *>(lds_raw);
  float *B = A + (kTileCells + 4) * P;
  float *HF = B + (kTileCells + 2) * P, *HC = HF + 8 * K, *HD = HC + 12 * N;
  const int W = (int)(blockDim.x >> 6);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const TileDev t = blk_desc<ARGT>(a, blockIdx.x);
  const bool hl = t.c0 > 0, hr = t.c0 + t.nc < a.J;   // halo cells (else ghost rows)
  // the halo cells' tables: issued first, stored to LDS with the rows
  constexpr int kHF = 4, kHC = 3;   // double2 load slots per thread (N <= 128)
  const int reg[2] = {hl ? a.cell_region[t.c0 - 1] : 0, hr ? a.cell_region[t.c0 + t.nc] : 0};
  const bool side_on[2] = {hl, hr};
  double2 hfv[kHF], hcv[kHC];
  float2 hdv = make_float2(0.f, 0.f);
#pragma unroll
  for (int i = 0; i < kHF; ++i) {   // H rows: 2K double2 per side
    const int e = threadIdx.x + i * (int)blockDim.x, sd = e / (2 * K), w = e - sd * 2 * K;
    hfv[i] = make_double2(0.0, 0.0);
    if (e < 4 * K && side_on[sd]) {
      const int q = w / (K / 2), kk = 2 * (w - q * (K / 2));
      hfv[i] = *reinterpret_cast<const double2 *>(a.phig + ((size_t)reg[sd] * 4 + q) * K + kk);
    }
  }
#pragma unroll
  for (int i = 0; i < kHC; ++i) {   // pair coefficients: 6 pairs x N/2 angles per side
    const int e = threadIdx.x + i * (int)blockDim.x, sd = e / (3 * N), w = e - sd * 3 * N;
    hcv[i] = make_double2(0.0, 0.0);
    if (e < 6 * N && side_on[sd]) {
      const int i2 = w / (N / 2), j = w - i2 * (N / 2);
      hcv[i] = coef_pair(a, N, reg[sd], sd == 0 ? N / 2 + j : j, i2);
    }
  }
  {   // defect pairs: N/2 per side
    const int e = threadIdx.x, sd = e / (N / 2), j = e - sd * (N / 2);
    if (e < N && side_on[sd]) {
      const int hc = sd == 0 ? t.c0 - 1 : t.c0 + t.nc, m = sd == 0 ? N / 2 + j : j;
      hdv = *reinterpret_cast<const float2 *>(a.dlt + (size_t)(hc + 1) * K + 2 * m);
    }
  }
  const float *src = a.dlt + (size_t)(n == 1 ? 0 : ((n & 1) ? 2 : 1)) * a.dlt_stride;
  float *dst = a.dlt + (size_t)((n & 1) ? 1 : 2) * a.dlt_stride;
  const float *dd = a.dlt;   // the defect d
  int prt, poff, kb, ke;
  phi_tile(N, &prt, &poff);
  phi_ksplit(KS, W, wave, &kb, &ke);
  const float *F = a.frag_it32 + (size_t)t.region * a.frag_it_stride + lane + (size_t)prt * KS * 64;
  const double *yb = nullptr, *ybp = nullptr;
  double *yo = nullptr, *yop = nullptr;
  int cur = 0, fb = 0;
  if (opens || ly == 2) {
    cur = a.ctl->cur;
    fb = a.ctl->fin_buf;
  }
  if (ly) {
    const int bb = ly == 2 ? fb : ring_buf(a, ly - 2, half);
    const int bo = ring_buf(a, ly, half);
    yb = out_at(a, bb);
    ybp = phi_at(a, bb);
    yo = out_at(a, bo);
    yop = phi_at(a, bo);
  }
  // loads that need no LDS: this wave's first operator fragments, this
  // thread's coefficients, the defect (and with ly the FP64 point) of its
  // first cells, and wave 0's scalar-flux defect (and FP64 point)
  float f0[kFr];
#pragma unroll
  for (int q = 0; q < kFr; ++q) f0[q] = F[(size_t)min(kb + q, KS - 1) * 64];
  const PairMap pm(N);
  float cf[12];
  {
    double c[12];
    coef_load<12>(a, N, t.region, pm.m, 0, c);
#pragma unroll
    for (int q = 0; q < 12; ++q) cf[q] = (float)c[q];
  }
  float dq[kDPre][2];
  double yq[kDPre][2];
#pragma unroll
  for (int j = 0; j < kDPre; ++j) {
    const size_t cell = (size_t)(t.c0 + min(pm.cl0 + j * pm.cstep, t.nc - 1));
    const float2 v = *reinterpret_cast<const float2 *>(dd + (cell + 1) * K + 2 * pm.m);
    dq[j][0] = v.x;
    dq[j][1] = v.y;
    yq[j][0] = yq[j][1] = 0.0;
    if (ly) {
      const double2 y = *reinterpret_cast<const double2 *>(yb + (cell + 1) * K + 2 * pm.m);
      yq[j][0] = y.x;
      yq[j][1] = y.y;
    }
  }
  float dphi = 0.f;
  double yphi = 0.0;
  if (wave == 0) {
    const size_t ce = (size_t)(t.c0 + min(lane >> 2, t.nc - 1)) * 4 + (lane & 3);
    dphi = a.dphi32[ce];
    if (ly) yphi = ybp[ce];
  }
  const int stalled = a.ctl->stalled;
  // rows of delta_i of cells c0-2 .. c0+nc+1 (ghosted rows c0-1 .. c0+nc+2,
  // clamped to the mesh) into block A
  const int g_lo = max(t.c0 - 1, 0), g_hi = min(t.c0 + t.nc + 2, a.J + 1);
  const int r_lo = g_lo - (t.c0 - 1);
  {
    const f4 *s4 = reinterpret_cast<const f4 *>(src + (size_t)g_lo * K);
    const int n4 = (g_hi - g_lo + 1) * K4;
    for (int e = threadIdx.x; e < n4; e += blockDim.x) {
      const int r = e / K4, k4 = e - r * K4;
      *reinterpret_cast<f4 *>(A + (r_lo + r) * P + 4 * k4) = s4[e];
    }
  }
#pragma unroll
  for (int i = 0; i < kHF; ++i) {
    const int e = threadIdx.x + i * (int)blockDim.x;
    if (e < 4 * K) {   // (side sd, row q, column kk) -> HF[sd][q][kk]: the same flat order
      HF[2 * e] = (float)hfv[i].x;
      HF[2 * e + 1] = (float)hfv[i].y;
    }
  }
#pragma unroll
  for (int i = 0; i < kHC; ++i) {
    const int e = threadIdx.x + i * (int)blockDim.x, sd = e / (3 * N), w = e - sd * 3 * N;
    if (e < 6 * N) {
      const int i2 = w / (N / 2), j = w - i2 * (N / 2);
      HC[(sd * 12 + 2 * i2) * (N / 2) + j] = (float)hcv[i].x;
      HC[(sd * 12 + 2 * i2 + 1) * (N / 2) + j] = (float)hcv[i].y;
    }
  }
  if (threadIdx.x < N) {
    HD[2 * threadIdx.x] = hdv.x;
    HD[2 * threadIdx.x + 1] = hdv.y;
  }
  __syncthreads();
  if (stalled) return;
  const bool refl = a.bcl == kBcReflect, refr = a.bcr == kBcReflect;
  // reflecting edges: the ghost next to a halo cell on the edge, or next to
  // the tile's own edge cell (the correction obeys the homogeneous mirror map)
  if (refl && t.c0 == 1) mirror_row32(A, A + P, N, true);
  if (refl && t.c0 == 0) mirror_row32(A + P, A + 2 * P, N, true);
  if (refr && t.c0 + t.nc == a.J - 1) mirror_row32(A + (t.nc + 3) * P, A + (t.nc + 2) * P, N, false);
  if (refr && t.c0 + t.nc == a.J) mirror_row32(A + (t.nc + 2) * P, A + (t.nc + 1) * P, N, false);
  if (refl || refr) __syncthreads();
  // level 1: the halo cells' entering pairs (one wave each) into block B
  const int wl = W - 1, wr = W >= 2 ? W - 2 : W - 1;
  for (int side = 0; side < 2; ++side) {
    const bool left = side == 0;
    if (!(left ? hl && wave == wl : hr && wave == wr)) continue;
    const float *row_l = A + (left ? 0 : t.nc + 1) * P;   // the halo cell's left neighbour
    const float *row_r = A + (left ? 2 : t.nc + 3) * P;   // and its right one
    float *orow = B + (left ? 0 : t.nc + 1) * P;
    const int q = lane >> 4;   // row q of the wave forms component q
    const float *Fq = HF + (side * 4 + q) * K;
    double acc = 0.0;
    for (int k = lane & 15; k < K; k += 16) acc += (double)(Fq[k] * (k < N ? row_r[k] : row_l[k]));
    acc = row_sum16(acc);
    float eh[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) eh[c] = (float)lane_f64(acc, 16 * c);
    const float *hcs = HC + side * 12 * (N / 2), *hds = HD + side * N;
    for (int j = lane; j < N / 2; j += 64) {
      const int m = left ? N / 2 + j : j;   // the angles entering the tile
      float c[12];
#pragma unroll
      for (int u = 0; u < 12; ++u) c[u] = hcs[u * (N / 2) + j];
      const float *in = (left ? row_l : row_r) + 2 * m;
      const float i0 = in[0], i1 = in[1];
      orow[2 * m] = hds[2 * j] + c[0] * eh[0] + c[1] * eh[1] + c[2] * eh[2] + c[3] * eh[3] +
                    c[4] * i0 + c[5] * i1;
      orow[2 * m + 1] = hds[2 * j + 1] + c[6] * eh[0] + c[7] * eh[1] + c[8] * eh[2] +
                        c[9] * eh[3] + c[10] * i0 + c[11] * i1;
    }
  }
  // level 1, own cells: e, then the full rows into block B (row cl + 1)
  inner_phi(A + P, P, KS, kb, ke, F, f0, phis32, ef);
  const int m = pm.m;
  const bool pos = 2 * m >= N;
  auto own_d = [&](int j, size_t cell, float &d0, float &d1) {
    if (j < kDPre) {   // (entry j by selects: a run-time index would put dq in scratch)
      d0 = dq[0][0];
      d1 = dq[0][1];
#pragma unroll
      for (int q = 1; q < kDPre; ++q)
        if (q == j) {
          d0 = dq[q][0];
          d1 = dq[q][1];
        }
    } else {
      d0 = dd[(cell + 1) * K + 2 * m];
      d1 = dd[(cell + 1) * K + 2 * m + 1];
    }
  };
  {
    int j = 0;
    for (int cl = pm.active ? pm.cl0 : t.nc; cl < t.nc; cl += pm.cstep, ++j) {
      const float *in = A + (pos ? cl + 1 : cl + 3) * P + 2 * m;
      const float *e4 = ef + cl * 4;
      float d0, d1;
      own_d(j, (size_t)(t.c0 + cl), d0, d1);
      const float i0 = in[0], i1 = in[1];
      const float e0 = e4[0], e1 = e4[1], e2 = e4[2], e3 = e4[3];
      B[(cl + 1) * P + 2 * m] = d0 + cf[0] * e0 + cf[1] * e1 + cf[2] * e2 + cf[3] * e3 +
                                cf[4] * i0 + cf[5] * i1;
      B[(cl + 1) * P + 2 * m + 1] = d1 + cf[6] * e0 + cf[7] * e1 + cf[8] * e2 + cf[9] * e3 +
                                    cf[10] * i0 + cf[11] * i1;
    }
  }
  __syncthreads();
  // ghost rows of block B at the mesh edges: zero, or the mirror of the edge
  // cell's delta_{i+1}
  if (!hl) {
    if (refl) mirror_row32(B, B + P, N, true);
    else for (int i = N + threadIdx.x; i < K; i += blockDim.x) B[i] = 0.f;
  }
  if (!hr) {
    float *g = B + (t.nc + 1) * P;
    if (refr) mirror_row32(g, B + t.nc * P, N, false);
    else for (int i = threadIdx.x; i < N; i += blockDim.x) g[i] = 0.f;
  }
  if (!hl || !hr) __syncthreads();
  // level 2: delta_{i+2} of the own cells from block B
  inner_phi(B, P, KS, kb, ke, F, f0, phis32, ef);
  if (ly && wave == 0) {
    const int cl = lane >> 2;
    if (cl < t.nc) yop[(size_t)(t.c0 + cl) * 4 + (lane & 3)] = yphi + (double)(dphi + ef[lane]);
  }
  int j = 0;
  for (int cl = pm.active ? pm.cl0 : t.nc; cl < t.nc; cl += pm.cstep, ++j) {
    const float *in = B + (pos ? cl : cl + 2) * P + 2 * m;
    const float *e4 = ef + cl * 4;
    const size_t cell = (size_t)(t.c0 + cl);
    float d0, d1;
    own_d(j, cell, d0, d1);
    const float i0 = in[0], i1 = in[1];
    const float e0 = e4[0], e1 = e4[1], e2 = e4[2], e3 = e4[3];
    const float o0 = d0 + cf[0] * e0 + cf[1] * e1 + cf[2] * e2 + cf[3] * e3 + cf[4] * i0 +
                     cf[5] * i1;
    const float o1 = d1 + cf[6] * e0 + cf[7] * e1 + cf[8] * e2 + cf[9] * e3 + cf[10] * i0 +
                     cf[11] * i1;
    if (ly) {
      double y0 = 0.0, y1 = 0.0;
      if (j < kDPre) {
        y0 = yq[0][0];
        y1 = yq[0][1];
#pragma unroll
        for (int q = 1; q < kDPre; ++q)
          if (q == j) {
            y0 = yq[q][0];
            y1 = yq[q][1];
          }
      } else {
        y0 = yb[(cell + 1) * K + 2 * m];
        y1 = yb[(cell + 1) * K + 2 * m + 1];
      }
      *reinterpret_cast<double2 *>(yo + (cell + 1) * K + 2 * m) =
          make_double2(y0 + (double)o0, y1 + (double)o1);
    } else {
      *reinterpret_cast<float2 *>(dst + (cell + 1) * K + 2 * m) = make_float2(o0, o1);
    }
  }
  if (opens) open_step(a, 1, cur, fb, stalled, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Learned corrections inside the iteration
// ---------------------------------------------------------------------------
// The corrector's input for iterate l of the open step (l >= 3): per cell the
// two latest scalar-flux differences, x [ch][J] in FP32 (channels 0..3:
// phi^(l) - phi^(l-1), 4..7: phi^(l-1) - phi^(l-2)) and, with ch = 12, the
// latest difference extrapolated with the iteration's observed contraction,
// amp (phi^(l) - phi^(l-1)), amp = rho / (1 - rho) (channels 8..11: what the
// remaining error would be if every error component contracted at rho).  No
// scaling: the network is positively homogeneous.
__global__ __launch_bounds__(256) void k_learn_features(StepArgs a, int l, int half, int ch,
                                                        double amp, float *x) {
  const double *p0 = phi_at(a, ring_buf(a, l, half));
  const double *p1 = phi_at(a, ring_buf(a, l - 1, half));
  const double *p2 = phi_at(a, ring_buf(a, l - 2, half));
  const int n = a.J * 4;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    const int j = e >> 2, c = e & 3;
    const double v0 = p0[e], v1 = p1[e], v2 = p2[e];
    x[(size_t)c * a.J + j] = (float)(v0 - v1);
    x[(size_t)(4 + c) * a.J + j] = (float)(v1 - v2);
    if (ch == 12) x[(size_t)(8 + c) * a.J + j] = (float)(amp * (v0 - v1));
  }
}

// The corrected iterate l in place: the scalar flux phi + dphi (dphi = the
// corrector's output y [4][J]) and every outgoing flux moved by the isotropic
// angular flux of that change on its half cell and time level,
// dpsi = dphi / sum_m w_m (= dphi / 2): the slowly converging error of OCI in
// thin, scattering cells is the nearly isotropic scattering mode, and it
// lives in the incident fluxes the next iterate reads, so the correction is
// carried there (a scalar flux moved alone would be recomputed from the
// uncorrected incident fluxes and lost).  Angle m < N/2 leaves through the
// left half (components 0, 2 at levels k, k+1/2), m >= N/2 through the right
// (1, 3).  One thread per (cell, angle).
__global__ __launch_bounds__(256) void k_learn_apply(StepArgs a, int l, int half, const float *y) {
  const int N = a.N, K = 2 * N;
  const int b = ring_buf(a, l, half);
  double *out = out_at(a, b), *phi = phi_at(a, b);
  const size_t n = (size_t)a.J * N;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(e / N), m = (int)(e - (size_t)j * N);
    const int side = 2 * m >= N ? 1 : 0;
    const double d0 = (double)y[(size_t)side * a.J + j];         // level k
    const double d1 = (double)y[(size_t)(2 + side) * a.J + j];   // level k+1/2
    double *o = out + (size_t)(j + 1) * K + 2 * m;
    o[0] += 0.5 * d0;
    o[1] += 0.5 * d1;
    if (m == 0) {
#pragma unroll
      for (int c = 0; c < 4; ++c) phi[(size_t)j * 4 + c] += (double)y[(size_t)c * a.J + j];
    }
  }
}

// ---------------------------------------------------------------------------
// Ensembles: one launch over the tiles of many problems
// ---------------------------------------------------------------------------
// A work queue of (problem, tile) entries (tile = the problem's tile count:
// its residual-reduction work-group) replaces blockIdx.x; every problem keeps
// its own argument block (probs[problem], in device memory), rings, records
// and control block, so each problem's iterates, decisions and end of step
// are those of its own launches.  Built for the common angle counts (NF =
// 8 .. 128, the work-group size of that N's own kernels) and for any N (NF =
// 0, a multiple of 8, 256 threads per work-group); one launch per angle count
// and launch shape (iterates per launch) covers all its problems.

// A pointer to device global memory, marked as such: accesses through it
// compile to global instructions instead of flat ones, which also count
// against the LDS wait counter, so that every wait for LDS data would wait
// for them too.  (An integer round trip: the compiler folds a plain
// generic -> global -> generic cast pair back to the generic pointer.)
template <class T>
__device__ __forceinline__ T *glob(T *p) {
  return (T *)(__attribute__((address_space(1))) T *)(uintptr_t)p;
}

// Problem p's argument block, copied out of device memory with every pointer
// marked as global memory (a kernel's own argument block is a kernel argument,
// whose pointers the compiler already knows to be global).
__device__ __forceinline__ StepArgs load_args(const StepArgs *__restrict__ probs, int p) {
  StepArgs a = probs[p];
  a.tiles = glob(a.tiles);
  a.frag_it = glob(a.frag_it);
  a.frag_pv = glob(a.frag_pv);
  a.c_pv = glob(a.c_pv);
  a.regions = glob(a.regions);
  a.mu = glob(a.mu);
  a.ainv = glob(a.ainv);
  a.coef = glob(a.coef);
  a.phig = glob(a.phig);
  a.cell_region = glob(a.cell_region);
  a.gh = glob(a.gh);
  a.outb = glob(a.outb);
  a.phib = glob(a.phib);
  a.psi0 = glob(a.psi0);
  a.psi1 = glob(a.psi1);
  a.phi_res = glob(a.phi_res);
  a.partial = glob(a.partial);
  a.dec = glob(a.dec);
  a.ctl = glob(a.ctl);
  a.rec = glob(a.rec);
  a.frag_it32 = glob(a.frag_it32);
  a.dlt = glob(a.dlt);
  a.dphi32 = glob(a.dphi32);
  return a;
}

template <int CH, int NF>
__global__ __launch_bounds__(256) void kb_step_begin(const StepArgs *__restrict__ probs,
                                                     const int2 *__restrict__ queue) {
  extern __shared__ double lds[];
  const int2 q = queue[blockIdx.x];
  const StepArgs a = load_args(probs, q.x);
  step_begin_body<CH, false, true, NF>(a, q.y, lds);
}

// (first[problem] .. last[problem]: the iterates planned for the problem in
// this batch; launch `node` computes iterate first + node - 1, and the
// launches past last leave the problem's work-groups idle)
template <int CH, int NF>
__global__ __launch_bounds__(256, 3) void kb_oci_iterate(const StepArgs *__restrict__ probs,
                                                         const int2 *__restrict__ queue,
                                                         const int *__restrict__ first,
                                                         const int *__restrict__ last, int node,
                                                         int half) {
  extern __shared__ double lds[];
  const int2 q = queue[blockIdx.x];
  const int cb = first[q.x] - 1;
  if (cb + node > last[q.x]) return;
  const StepArgs a = load_args(probs, q.x);
  oci_iterate_body<CH, false, true, NF>(a, q.y, lds, node, cb, half, 1, 1);
}

// Launches every KI nodes (1, 1 + KI, ...): each computes up to KI of the
// problem's iterates, fewer at the end of its range, and its reduction
// work-group reduces the KI iterates of the problem's launch before (none at
// node 1: the iterates before first are reduced already).
template <int CH, int NF, int KI>
__global__ __launch_bounds__(256, 2) void kb_oci_iterateK(const StepArgs *__restrict__ probs,
                                                          const int2 *__restrict__ queue,
                                                          const int *__restrict__ first,
                                                          const int *__restrict__ last, int node,
                                                          int half) {
  const int2 q = queue[blockIdx.x];
  const int f = first[q.x];
  const int kk = ocip::ens_levels(f, last[q.x], node, KI);
  if (kk <= 0) return;
  const StepArgs a = load_args(probs, q.x);
  oci_iterateK_body<CH, false, true, NF, KI>(a, q.y, node, f - 1, half,
                                             ocip::ens_reduced_before(node, KI), kk);
}

// (one work-group per listed problem: the iterates of its last launch,
// (last - first) mod ki + 1 of them)
__global__ __launch_bounds__(256) void kb_reduce_rec(const StepArgs *__restrict__ probs,
                                                     const int *__restrict__ plist,
                                                     const int *__restrict__ first,
                                                     const int *__restrict__ last,
                                                     const int *__restrict__ ki, int half) {
  const int p = plist[blockIdx.x];
  const StepArgs a = load_args(probs, p);
  reduce_rec_body(a, last[p], ocip::ens_trailing(first[p], last[p], ki[p]), half);
}

template <int CH, int NF>
__global__ __launch_bounds__(256, 3) void kb_step_end(const StepArgs *__restrict__ probs,
                                                      double *const *__restrict__ phi_outs,
                                                      const int2 *__restrict__ queue,
                                                      const int *__restrict__ first,
                                                      const int *__restrict__ last, int half,
                                                      int mode) {
  extern __shared__ double lds[];
  const int2 q = queue[blockIdx.x];
  const StepArgs a = load_args(probs, q.x);
  step_end_body<CH, false, true, NF, false>(a, q.y, lds,
                                            phi_outs ? glob(phi_outs[q.x]) : nullptr, first[q.x],
                                            last[q.x], half, 1, mode);
}

// Control blocks of the listed problems (one thread each).
__global__ __launch_bounds__(256) void kb_set_ctl(const StepArgs *probs, const int *plist, int n,
                                                  int psi_base) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= n) return;
  StepCtl *c = probs[plist[i]].ctl;
  if (psi_base >= 0) {
    c->cur = 0;
    c->psi_base = psi_base;
  } else {
    c->stalled = 0;
  }
}

#define OCI_KB(CHV, NFV)                                                                      \
  template __global__ void kb_step_begin<CHV, NFV>(const StepArgs *, const int2 *);           \
  template __global__ void kb_oci_iterate<CHV, NFV>(const StepArgs *, const int2 *,           \
                                                    const int *, const int *, int, int);      \
  template __global__ void kb_step_end<CHV, NFV>(const StepArgs *, double *const *,           \
                                                 const int2 *, const int *, const int *, int, \
                                                 int);
OCI_KB(4, 0)
OCI_KB(4, 8)
OCI_KB(8, 16)
OCI_KB(16, 32)
OCI_KB(16, 64)
OCI_KB(16, 128)
#undef OCI_KB
#define OCI_KBK(CHV, NFV, KIV)                                                        \
  template __global__ void kb_oci_iterateK<CHV, NFV, KIV>(const StepArgs *, const int2 *, \
                                                          const int *, const int *, int, int);
OCI_KBK(4, 8, 3)
OCI_KBK(4, 8, 4)
OCI_KBK(8, 16, 3)
OCI_KBK(8, 16, 4)
OCI_KBK(16, 32, 3)
OCI_KBK(16, 32, 4)
OCI_KBK(16, 64, 3)
OCI_KBK(16, 64, 4)
#undef OCI_KBK

template __global__ void k_oci_iterate2<4, false, false, 0>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterate2<4, false, true, 0>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterate2<8, false, false, 0>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterate2<8, false, true, 0>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterate2<16, false, false, 0>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterate2<16, false, true, 0>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterate2<4, false, true, 8>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterate2<8, false, true, 16>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterate2<16, false, true, 32>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterate2<16, false, true, 64>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterate2<16, false, true, 128>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterate2<16, false, true, 256>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterate2<4, true, false, 0>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterate2<4, true, true, 0>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterate2<8, true, false, 0>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterate2<8, true, true, 0>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterate2<16, true, false, 0>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterate2<16, true, true, 0>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterate2<4, true, true, 8>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterate2<8, true, true, 16>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterate2<16, true, true, 32>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterate2<16, true, true, 64>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterate2<16, true, true, 128>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterate2<16, true, true, 256>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterateK<4, true, true, 8, 3>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterateK<8, true, true, 16, 3>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterateK<16, true, true, 32, 3>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterateK<4, false, true, 8, 3>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterateK<8, false, true, 16, 3>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterateK<16, false, true, 32, 3>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterateK<4, true, true, 8, 4>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterateK<8, true, true, 16, 4>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterateK<16, true, true, 32, 4>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterateK<4, false, true, 8, 4>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterateK<8, false, true, 16, 4>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterateK<16, false, true, 32, 4>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterateK<16, true, true, 64, 3>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterateK<16, false, true, 64, 3>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterateK<16, true, true, 64, 4>(StepArgs, int, int, int, int);
template __global__ void k_oci_iterateK<16, false, true, 64, 4>(StepArgs, int, int, int, int);
template __global__ void k_oci_inner<true>(StepArgs, int, int, int, int);
template __global__ void k_oci_inner<false>(StepArgs, int, int, int, int);
template __global__ void k_oci_inner2<true>(StepArgs, int, int, int, int);
template __global__ void k_oci_inner2<false>(StepArgs, int, int, int, int);

template __global__ void k_step_begin<4, false, false, 0>(StepArgs);
template __global__ void k_oci_iterate<4, false, false, 0>(StepArgs, int, int, int, int, int);
template __global__ void k_step_end<4, false, false, 0>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_end_nf<4, false, false, 0>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_begin<4, false, true, 0>(StepArgs);
template __global__ void k_oci_iterate<4, false, true, 0>(StepArgs, int, int, int, int, int);
template __global__ void k_step_end<4, false, true, 0>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_end_nf<4, false, true, 0>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_begin<8, false, false, 0>(StepArgs);
template __global__ void k_oci_iterate<8, false, false, 0>(StepArgs, int, int, int, int, int);
template __global__ void k_step_end<8, false, false, 0>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_end_nf<8, false, false, 0>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_begin<8, false, true, 0>(StepArgs);
template __global__ void k_oci_iterate<8, false, true, 0>(StepArgs, int, int, int, int, int);
template __global__ void k_step_end<8, false, true, 0>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_end_nf<8, false, true, 0>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_begin<16, false, false, 0>(StepArgs);
template __global__ void k_oci_iterate<16, false, false, 0>(StepArgs, int, int, int, int, int);
template __global__ void k_step_end<16, false, false, 0>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_end_nf<16, false, false, 0>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_begin<16, false, true, 0>(StepArgs);
template __global__ void k_oci_iterate<16, false, true, 0>(StepArgs, int, int, int, int, int);
template __global__ void k_step_end<16, false, true, 0>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_end_nf<16, false, true, 0>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_begin<4, false, true, 8>(StepArgs);
template __global__ void k_oci_iterate<4, false, true, 8>(StepArgs, int, int, int, int, int);
template __global__ void k_step_end<4, false, true, 8>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_end_nf<4, false, true, 8>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_begin<8, false, true, 16>(StepArgs);
template __global__ void k_oci_iterate<8, false, true, 16>(StepArgs, int, int, int, int, int);
template __global__ void k_step_end<8, false, true, 16>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_end_nf<8, false, true, 16>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_begin<16, false, true, 32>(StepArgs);
template __global__ void k_oci_iterate<16, false, true, 32>(StepArgs, int, int, int, int, int);
template __global__ void k_step_end<16, false, true, 32>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_end_nf<16, false, true, 32>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_begin<16, false, true, 64>(StepArgs);
template __global__ void k_oci_iterate<16, false, true, 64>(StepArgs, int, int, int, int, int);
template __global__ void k_step_end<16, false, true, 64>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_end_nf<16, false, true, 64>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_begin<16, false, true, 128>(StepArgs);
template __global__ void k_oci_iterate<16, false, true, 128>(StepArgs, int, int, int, int, int);
template __global__ void k_step_end<16, false, true, 128>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_end_nf<16, false, true, 128>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_begin<16, false, true, 256>(StepArgs);
template __global__ void k_oci_iterate<16, false, true, 256>(StepArgs, int, int, int, int, int);
template __global__ void k_step_end<16, false, true, 256>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_end_nf<16, false, true, 256>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_begin<4, true, false, 0>(StepArgs);
template __global__ void k_oci_iterate<4, true, false, 0>(StepArgs, int, int, int, int, int);
template __global__ void k_step_end<4, true, false, 0>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_end_nf<4, true, false, 0>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_begin<4, true, true, 0>(StepArgs);
template __global__ void k_oci_iterate<4, true, true, 0>(StepArgs, int, int, int, int, int);
template __global__ void k_step_end<4, true, true, 0>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_end_nf<4, true, true, 0>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_begin<8, true, false, 0>(StepArgs);
template __global__ void k_oci_iterate<8, true, false, 0>(StepArgs, int, int, int, int, int);
template __global__ void k_step_end<8, true, false, 0>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_end_nf<8, true, false, 0>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_begin<8, true, true, 0>(StepArgs);
template __global__ void k_oci_iterate<8, true, true, 0>(StepArgs, int, int, int, int, int);
template __global__ void k_step_end<8, true, true, 0>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_end_nf<8, true, true, 0>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_begin<16, true, false, 0>(StepArgs);
template __global__ void k_oci_iterate<16, true, false, 0>(StepArgs, int, int, int, int, int);
template __global__ void k_step_end<16, true, false, 0>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_end_nf<16, true, false, 0>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_begin<16, true, true, 0>(StepArgs);
template __global__ void k_oci_iterate<16, true, true, 0>(StepArgs, int, int, int, int, int);
template __global__ void k_step_end<16, true, true, 0>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_end_nf<16, true, true, 0>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_begin<4, true, true, 8>(StepArgs);
template __global__ void k_oci_iterate<4, true, true, 8>(StepArgs, int, int, int, int, int);
template __global__ void k_step_end<4, true, true, 8>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_end_nf<4, true, true, 8>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_begin<8, true, true, 16>(StepArgs);
template __global__ void k_oci_iterate<8, true, true, 16>(StepArgs, int, int, int, int, int);
template __global__ void k_step_end<8, true, true, 16>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_end_nf<8, true, true, 16>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_begin<16, true, true, 32>(StepArgs);
template __global__ void k_oci_iterate<16, true, true, 32>(StepArgs, int, int, int, int, int);
template __global__ void k_step_end<16, true, true, 32>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_end_nf<16, true, true, 32>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_begin<16, true, true, 64>(StepArgs);
template __global__ void k_oci_iterate<16, true, true, 64>(StepArgs, int, int, int, int, int);
template __global__ void k_step_end<16, true, true, 64>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_end_nf<16, true, true, 64>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_begin<16, true, true, 128>(StepArgs);
template __global__ void k_oci_iterate<16, true, true, 128>(StepArgs, int, int, int, int, int);
template __global__ void k_step_end<16, true, true, 128>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_end_nf<16, true, true, 128>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_begin<16, true, true, 256>(StepArgs);
template __global__ void k_oci_iterate<16, true, true, 256>(StepArgs, int, int, int, int, int);
template __global__ void k_step_end<16, true, true, 256>(StepArgs, double *, int, int, int, int, int);
template __global__ void k_step_end_nf<16, true, true, 256>(StepArgs, double *, int, int, int, int, int);

}  // namespace ocik
