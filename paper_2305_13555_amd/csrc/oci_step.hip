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
#include "oci_kernels.h"

namespace ocik {


// Work-group index -> tile: consecutive tiles go to the same XCD (work-groups
// are dispatched round-robin over the 8 XCDs), so a region's operator is
// read into few L2s.  The grid has 8*ceil(ntiles/8) work-groups, on which
// this map is a bijection; the surplus ones get -1 and exit.
__device__ __forceinline__ int tile_of_block(int b, int ntiles) {
  const int nx = 8;
  const int per = (ntiles + nx - 1) / nx;
  const int t = (b % nx) * per + b / nx;
  return t < ntiles ? t : -1;
}

// Stage the outgoing rows of cells c0-1 .. c0+nc (ghosted rows c0 .. c0+nc+1)
// into LDS rows 0 .. nc+1 (pitch P), zero elsewhere up to row 17, then apply
// reflecting edges: the ghost takes the boundary cell's mirror-angle values.
__device__ inline void stage_neighbours(double *lds, int P, const double *src, const TileDev &t,
                                        int N, int J, int bcl, int bcr) {
  const int K = 2 * N;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, W = blockDim.x >> 6;
  for (int r = wave; r < kTileCells + 2; r += W) {
    const bool live = r <= t.nc + 1;
    const double *g = src + (size_t)(t.c0 + r) * K;
    for (int k = lane; k < K; k += kWave) lds[r * P + k] = live ? g[k] : 0.0;
  }
  __syncthreads();
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

// ---------------------------------------------------------------------------
// Per-step constant: gh_j = P_r psi_{k-1/2,j} + p_r; resets the step state.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(512) void k_step_begin(StepArgs a) {
  extern __shared__ double lds[];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    StepState *st = a.st;
    st->it = 0;
    st->done = kRunning;
    st->arrive = 0;
    st->step_parity = a.step_parity;
    st->e_last = -1.0;
    st->e_prev = -1.0;
  }
  const int ti = tile_of_block(blockIdx.x, a.ntiles);
  if (ti < 0) return;
  const TileDev t = a.tiles[ti];
  const int N = a.N, K = 2 * N, P = K + 2;
  const double *psi_prev = a.step_parity ? a.psi1 : a.psi0;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, W = blockDim.x >> 6;
  for (int r = wave; r < kTileCells; r += W) {
    const bool live = r < t.nc;
    const double *g = psi_prev + (size_t)(t.c0 + r) * K;
    for (int k = lane; k < K; k += kWave) lds[r * P + k] = live ? g[k] : 0.0;
  }
  __syncthreads();
  const int col = lane & 15, kq = lane >> 4;
  const int KS = K / 4;
  const double *F = a.frag_pv + (size_t)t.region * a.frag_pv_stride;
  const double *cp = a.c_pv + (size_t)t.region * a.c_pv_stride;
  const double *arow = lds + col * P + kq;
  const int ghp = a.Mt * 16;
  for (int rt = wave; rt < a.Mt; rt += W) {
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    const double *Fr = F + (size_t)rt * KS * 64 + lane;
    for (int ks = 0; ks < KS; ++ks) acc = mfma16x16x4(arow[ks * 4], Fr[ks * 64], acc);
    const int row = rt * 16 + col;      // output row of this lane
    const double cv = cp[row];
    for (int i = 0; i < 4; ++i) {
      const int cl = kq + 4 * i;        // cell of element i
      if (cl < t.nc) a.gh[(size_t)(t.c0 + cl) * ghp + row] = acc[i] + cv;
    }
  }
}

// ---------------------------------------------------------------------------
// One OCI iteration over every cell (launched once per iteration; a no-op
// once the step is decided).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(512) void k_oci_iterate(StepArgs a) {
  extern __shared__ double lds[];
  StepState *st = a.st;
  const int done = st->done;
  const int it = st->it;
  if (done != kRunning || it >= a.max_iters) return;
  const int total = st->total;
  const double *src = (total & 1) ? a.out1 : a.out0;
  double *dst = (total & 1) ? a.out0 : a.out1;
  const double *phi_old = (total & 1) ? a.phi1 : a.phi0;
  double *phi_new = (total & 1) ? a.phi0 : a.phi1;

  const int ti = tile_of_block(blockIdx.x, a.ntiles);
  if (ti < 0) return;
  const TileDev t = a.tiles[ti];
  const int N = a.N, K = 2 * N, P = K + 2;
  stage_neighbours(lds, P, src, t, N, a.J, a.bcl, a.bcr);

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, W = blockDim.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const int KS = K / 4;
  const double *F = a.frag_it + (size_t)t.region * a.frag_it_stride;
  // incident flux of cell col, entry k: k < N from the right neighbour
  // (LDS row col+2), k >= N from the left neighbour (LDS row col)
  const double *a_lo = lds + (col + 2) * P + kq;
  const double *a_hi = lds + col * P + kq;
  const int ks_split = N / 4;          // k-steps entirely below N
  const int ghp = a.Mt * 16;
  const int rt_phi = K / 16;           // the row tile holding the phi rows
  const int owner = rt_phi % W;
  double dphi = 0.0, fphi = 0.0;
  int nonfinite = 0;
  for (int rt = wave; rt < a.Mt; rt += W) {
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    const double *Fr = F + (size_t)rt * KS * 64 + lane;
    int ks = 0;
    for (; ks < ks_split; ++ks) acc = mfma16x16x4(a_lo[ks * 4], Fr[ks * 64], acc);
    for (; ks < KS; ++ks) {
      const int k = ks * 4 + kq;
      const double av = k < N ? a_lo[ks * 4] : a_hi[ks * 4];
      acc = mfma16x16x4(av, Fr[ks * 64], acc);
    }
    const int row = rt * 16 + col;      // output row of this lane
    if (row < K + 4) {
      for (int i = 0; i < 4; ++i) {
        const int cl = kq + 4 * i;      // cell of element i
        if (cl >= t.nc) continue;
        const int cell = t.c0 + cl;
        const double v = acc[i] + a.gh[(size_t)cell * ghp + row];
        if (row < K) {
          dst[(size_t)(cell + 1) * K + row] = v;
        } else {
          const int c = row - K;
          const double o = phi_old[(size_t)cell * 4 + c];
          phi_new[(size_t)cell * 4 + c] = v;
          dphi = fmax(dphi, fabs(v - o));
          fphi = fmax(fphi, fabs(v));
          nonfinite |= !isfinite(v);
        }
      }
    }
  }
  if (wave != owner) return;
  // residual of this tile, then the last tile to finish decides the step
  dphi = wave_max(dphi);
  fphi = wave_max(fphi);
  nonfinite = wave_or(nonfinite);
  unsigned prev = 0;
  if (lane == 0) {
    double *pp = a.partial + (size_t)ti * 4;
    store_agent(pp + 0, dphi);
    store_agent(pp + 1, fphi);
    store_agent(pp + 2, (double)nonfinite);
    __threadfence();
    prev = atomicAdd(&st->arrive, 1u);
  }
  prev = __shfl(prev, 0, kWave);
  if (prev != (unsigned)(a.ntiles - 1)) return;
  __threadfence();
  double d = 0.0, f = 0.0, nf = 0.0;
  for (int i = lane; i < a.ntiles; i += kWave) {
    const double *pp = a.partial + (size_t)i * 4;
    d = fmax(d, load_agent(pp + 0));
    f = fmax(f, load_agent(pp + 1));
    nf = fmax(nf, load_agent(pp + 2));
  }
  d = wave_max(d);
  f = wave_max(f);
  nf = wave_max(nf);
  if (lane == 0) decide(st, d, f, nf != 0.0, a.max_iters, a.tol, a.strict, 2);
}

// ---------------------------------------------------------------------------
// End of step: psi_{k+1/2} from the incident fluxes of the accepted iterate
// (those the last iteration read) and psi_{k-1/2}; copies the accepted phi.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(512) void k_step_end(StepArgs a) {
  extern __shared__ double lds[];
  StepState *st = a.st;
  const int total = st->total;
  const double *src = (total & 1) ? a.out0 : a.out1;   // read by the last iteration
  const double *phi_acc = (total & 1) ? a.phi1 : a.phi0;
  const double *psi_prev = a.step_parity ? a.psi1 : a.psi0;
  double *psi_next = a.step_parity ? a.psi0 : a.psi1;
  const int ti = tile_of_block(blockIdx.x, a.ntiles);
  if (ti < 0) return;
  const TileDev t = a.tiles[ti];
  const int N = a.N, K = 2 * N, P = K + 2;
  double *ldp = lds + (kTileCells + 2) * P;
  stage_neighbours(lds, P, src, t, N, a.J, a.bcl, a.bcr);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, W = blockDim.x >> 6;
  for (int r = wave; r < kTileCells; r += W) {
    const bool live = r < t.nc;
    const double *g = psi_prev + (size_t)(t.c0 + r) * K;
    for (int k = lane; k < K; k += kWave) ldp[r * P + k] = live ? g[k] : 0.0;
  }
  for (int i = threadIdx.x; i < t.nc * 4; i += blockDim.x)
    a.phi_res[(size_t)t.c0 * 4 + i] = phi_acc[(size_t)t.c0 * 4 + i];
  __syncthreads();
  const int col = lane & 15, kq = lane >> 4;
  const int KS = (2 * K) / 4;
  const double *F = a.frag_ed + (size_t)t.region * a.frag_ed_stride;
  const double *ce = a.c_ed + (size_t)t.region * a.c_ed_stride;
  for (int rt = wave; rt < a.Met; rt += W) {
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    const double *Fr = F + (size_t)rt * KS * 64 + lane;
    for (int ks = 0; ks < KS; ++ks) {
      const int k = ks * 4 + kq;
      double av;
      if (k < N) av = lds[(col + 2) * P + k];
      else if (k < K) av = lds[col * P + k];
      else av = ldp[col * P + (k - K)];
      acc = mfma16x16x4(av, Fr[ks * 64], acc);
    }
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

}  // namespace ocik
