// Source iteration (Sec. "Source Iteration (SI)"): with the scalar flux of
// the previous iteration, every angle is swept through the mesh and each cell
// solves its 4x4 system A^+ x = b^+ (mu > 0) or A^- x = b^- (mu < 0).
//
// On the GPU a sweep is parallel over angles (mirror pairs m, N-1-m) and over
// cells by a two-level scan: with the lagged scalar flux fixed, the map from
// the flux entering a cell (levels k and k+1/2) to the flux leaving it is
// affine, x_out = T x_in + t, with T = |mu| (A^{-1})[out rows, in rows] and
// t = (A^{-1} b)[out rows] (the A_m^{-1} of the OCI setup, k_region_setup).
// The cells are split into S segments, one work-group per (pair, segment).  A first launch composes every segment's
// map (each thread a chunk of cells, a work-group scan of the chunk maps); a
// second gives every segment its entering flux from the maps upstream of it,
// and every thread re-sweeps its chunk from the entering flux the scan gives
// it.  The result is the sequential sweep up to rounding.
//
// Reflecting edges: the pair is swept in the order that makes the reflection
// exact within the iteration (mu < 0 first when the left edge reflects, mu > 0
// first when only the right edge reflects); with both edges reflecting the
// right edge uses the previous iteration's outgoing flux.
#include "oci_kernels.h"

namespace ocik {


// (f o g)(x) = f(g(x))
__device__ __forceinline__ Affine compose(const Affine &f, const Affine &g) {
  Affine r;
  r.m00 = f.m00 * g.m00 + f.m01 * g.m10;
  r.m01 = f.m00 * g.m01 + f.m01 * g.m11;
  r.m10 = f.m10 * g.m00 + f.m11 * g.m10;
  r.m11 = f.m10 * g.m01 + f.m11 * g.m11;
  r.v0 = f.m00 * g.v0 + f.m01 * g.v1 + f.v0;
  r.v1 = f.m10 * g.v0 + f.m11 * g.v1 + f.v1;
  return r;
}

// Local solve of cell j in angle m: y = A^{-1} b (b without the entering
// flux), plus the two columns of A^{-1} through which the entering flux acts.
struct CellSolve {
  double y[4];
  double c0[4], c1[4];   // |mu| * A^{-1}[:, in0], |mu| * A^{-1}[:, in1]
};

__device__ __forceinline__ CellSolve cell_solve(const SiArgs &a, const double *phi_old,
                                                const double *psi_prev, int j, int m, bool pos,
                                                double amu) {
  const int r = a.cell_region[j];
  const RegionDev g = a.regions[r];
  const double *Ai = a.ainv + ((size_t)r * a.N + m) * 16;
  const int K = 2 * a.N;
  double b[4];
  const double qs = g.dx / 4.0;
  for (int c = 0; c < 4; ++c) b[c] = qs * (g.sigs * phi_old[(size_t)j * 4 + c] + g.q);
  b[0] += a.a * g.dx / 2.0 * psi_prev[(size_t)j * K + 2 * m];
  b[1] += a.a * g.dx / 2.0 * psi_prev[(size_t)j * K + 2 * m + 1];
  CellSolve s;
  const int in0 = pos ? 0 : 1, in1 = pos ? 2 : 3;
  for (int i = 0; i < 4; ++i) {
    s.y[i] = Ai[i * 4 + 0] * b[0] + Ai[i * 4 + 1] * b[1] + Ai[i * 4 + 2] * b[2] + Ai[i * 4 + 3] * b[3];
    s.c0[i] = amu * Ai[i * 4 + in0];
    s.c1[i] = amu * Ai[i * 4 + in1];
  }
  return s;
}

__device__ __forceinline__ void apply(const Affine &f, double &x0, double &x1) {
  const double y0 = f.m00 * x0 + f.m01 * x1 + f.v0;
  const double y1 = f.m10 * x0 + f.m11 * x1 + f.v1;
  x0 = y0;
  x1 = y1;
}

// Cells of segment s of S: an even split of [0, J).
__device__ __forceinline__ int seg_edge(int s, int J, int S) {
  return (int)(((long long)J * s) / S);
}

// The two sweeps of angle pair p, in their order: pass 0 is mu < 0 unless
// only the right edge reflects.
__device__ __forceinline__ bool pass_positive(const SiArgs &a, int pass) {
  const bool pos_first = (a.bcr == kBcReflect && a.bcl != kBcReflect);
  return pos_first ? (pass == 0) : (pass == 1);
}

// This thread's chunk [jb, je) of segment [lo, hi), in cells.
__device__ __forceinline__ void chunk_of(int lo, int hi, int *jb, int *je) {
  const int n = hi - lo, C = (n + blockDim.x - 1) / blockDim.x;
  *jb = lo + min(n, (int)threadIdx.x * C);
  *je = lo + min(n, ((int)threadIdx.x + 1) * C);
}

// Map from the flux entering this thread's chunk to the flux leaving it, in
// sweep order.
__device__ Affine chunk_map(const SiArgs &a, const double *phi_old, const double *psi_prev,
                            int jb, int je, int m, bool pos) {
  const double amu = fabs(a.mu[m]);
  const int o0 = pos ? 1 : 0, o1 = pos ? 3 : 2;
  Affine f = {1.0, 0.0, 0.0, 1.0, 0.0, 0.0};
  for (int q = 0; q < je - jb; ++q) {
    const int j = pos ? jb + q : je - 1 - q;
    const CellSolve cs = cell_solve(a, phi_old, psi_prev, j, m, pos, amu);
    const Affine g = {cs.c0[o0], cs.c1[o0], cs.c0[o1], cs.c1[o1], cs.y[o0], cs.y[o1]};
    f = compose(g, f);
  }
  return f;
}

// Inclusive scan of the threads' chunk maps in sweep order (spos = position
// of this thread in that order); s_map[nt-1] is then the whole segment's map.
__device__ void scan_maps(Affine f, int spos, Affine *s_map) {
  const int nt = blockDim.x;
  s_map[spos] = f;
  __syncthreads();
  for (int off = 1; off < nt; off <<= 1) {
    const Affine mine = s_map[spos];
    Affine earlier = {1.0, 0.0, 0.0, 1.0, 0.0, 0.0};
    if (spos >= off) earlier = s_map[spos - off];
    __syncthreads();
    if (spos >= off) s_map[spos] = compose(mine, earlier);
    __syncthreads();
  }
}

constexpr int kSiThreads = 256;

// Sweep, first half: for iterate l = cb + node, the map of every segment of
// every angle pair, in both sweep directions (they depend only on the
// previous iterate's scalar flux and on psi_{k-1/2}).  Grid (N/2, S).
__global__ __launch_bounds__(kSiThreads) void k_si_maps(SiArgs a, int node, int cbase) {
  const StepCtl c = *a.ctl;
  if (c.stalled || c.status != kRunning) return;
  const int l = cbase + node;
  const double *phi_old = ((l - 1) & 1) ? a.phi1 : a.phi0;
  const double *psi_prev = c.step_parity ? a.psi1 : a.psi0;
  const int p = blockIdx.x, s = blockIdx.y, S = gridDim.y;
  const int lo = seg_edge(s, a.J, S), hi = seg_edge(s + 1, a.J, S);
  int jb, je;
  chunk_of(lo, hi, &jb, &je);
  __shared__ Affine s_map[kSiThreads];
  for (int pass = 0; pass < 2; ++pass) {
    const bool pos = pass_positive(a, pass);
    const int m = pos ? a.N - 1 - p : p;
    const Affine f = chunk_map(a, phi_old, psi_prev, jb, je, m, pos);
    const int spos = pos ? threadIdx.x : blockDim.x - 1 - threadIdx.x;
    scan_maps(f, spos, s_map);
    if (threadIdx.x == 0) a.segmap[((size_t)p * S + s) * 2 + pass] = s_map[blockDim.x - 1];
    __syncthreads();
  }
}

// Sweep, second half: every segment gets its entering flux from the maps of
// the segments upstream of it (applied to the flux entering the domain; the
// second direction starts from the first one's leaving flux where the edge
// reflects), then every thread re-sweeps its chunk from the flux the scan of
// the chunk maps gives it, writing the pair's contribution to the scalar
// flux, psi_{k+1/2} and the outgoing fluxes.  Grid (N/2, S).
__global__ __launch_bounds__(kSiThreads) void k_si_sweep(SiArgs a, int node, int cbase) {
  const StepCtl c = *a.ctl;
  if (c.stalled || c.status != kRunning) return;
  const int l = cbase + node;
  const int par = (l - 1) & 1;
  const int parity = c.step_parity;
  const double *phi_old = par ? a.phi1 : a.phi0;
  double *out_dst = par ? a.out0 : a.out1;
  const double *ghosts = a.out0;   // ghost rows are identical in both buffers
  const double *psi_prev = parity ? a.psi1 : a.psi0;
  double *psi_next = parity ? a.psi0 : a.psi1;
  const double *lag_in = a.lag + (size_t)par * a.N;
  double *lag_out = a.lag + (size_t)(l & 1) * a.N;
  const int N = a.N, J = a.J, K = 2 * N;
  const int p = blockIdx.x, s = blockIdx.y, S = gridDim.y;
  const int lo = seg_edge(s, J, S), hi = seg_edge(s + 1, J, S);
  int jb, je;
  chunk_of(lo, hi, &jb, &je);
  const Affine *maps = a.segmap + (size_t)p * S * 2;
  __shared__ Affine s_map[kSiThreads];
  __shared__ double s_in[2][2];
  if (threadIdx.x == 0) {
    // flux entering the domain and this segment, both passes
    double exit0 = 0.0, exit1 = 0.0;   // pass 0's leaving flux at its far edge
    for (int pass = 0; pass < 2; ++pass) {
      const bool pos = pass_positive(a, pass);
      const int m = pos ? N - 1 - p : p;
      double x0 = 0.0, x1 = 0.0;
      if (pos) {
        if (pass == 1 && a.bcl == kBcReflect) { x0 = exit0; x1 = exit1; }
        else if (a.bcl == kBcIncident) { x0 = ghosts[2 * m]; x1 = ghosts[2 * m + 1]; }
      } else {
        if (a.bcr == kBcReflect) {
          if (pass == 1) { x0 = exit0; x1 = exit1; }
          else { x0 = lag_in[2 * p]; x1 = lag_in[2 * p + 1]; }   // both edges reflect
        } else if (a.bcr == kBcIncident) {
          const double *gr = ghosts + (size_t)(J + 1) * K;
          x0 = gr[2 * m];
          x1 = gr[2 * m + 1];
        }
      }
      // segments in sweep order: ascending for mu > 0, descending for mu < 0
      for (int q = 0; q < S; ++q) {
        const int t = pos ? q : S - 1 - q;
        if (t == s) {
          s_in[pass][0] = x0;
          s_in[pass][1] = x1;
        }
        apply(maps[t * 2 + pass], x0, x1);
      }
      if (pass == 0) {
        exit0 = x0;
        exit1 = x1;
      } else if (a.bcl == kBcReflect && a.bcr == kBcReflect && s == 0) {
        // mu > 0 was swept second: its leaving flux at x = X is the next
        // iteration's entering flux of the mirror angle
        lag_out[2 * p] = x0;
        lag_out[2 * p + 1] = x1;
      }
    }
  }
  __syncthreads();
  double *contrib = a.contrib + (size_t)p * J * 4;
  for (int pass = 0; pass < 2; ++pass) {
    const bool pos = pass_positive(a, pass);
    const int m = pos ? N - 1 - p : p;
    const double amu = fabs(a.mu[m]), wm = a.w[m];
    const int o0 = pos ? 1 : 0, o1 = pos ? 3 : 2;
    const Affine f = chunk_map(a, phi_old, psi_prev, jb, je, m, pos);
    const int spos = pos ? threadIdx.x : blockDim.x - 1 - threadIdx.x;
    scan_maps(f, spos, s_map);
    double x0 = s_in[pass][0], x1 = s_in[pass][1];
    if (spos > 0) apply(s_map[spos - 1], x0, x1);
    for (int q = 0; q < je - jb; ++q) {
      const int j = pos ? jb + q : je - 1 - q;
      const CellSolve cs = cell_solve(a, phi_old, psi_prev, j, m, pos, amu);
      double x[4];
      for (int i = 0; i < 4; ++i) x[i] = cs.y[i] + cs.c0[i] * x0 + cs.c1[i] * x1;
      double *cj = contrib + (size_t)j * 4;
      if (pass == 0) {
        for (int i = 0; i < 4; ++i) cj[i] = wm * x[i];
      } else {
        for (int i = 0; i < 4; ++i) cj[i] += wm * x[i];
      }
      psi_next[(size_t)j * K + 2 * m] = x[2];
      psi_next[(size_t)j * K + 2 * m + 1] = x[3];
      out_dst[(size_t)(j + 1) * K + 2 * m] = x[o0];
      out_dst[(size_t)(j + 1) * K + 2 * m + 1] = x[o1];
      x0 = x[o0];
      x1 = x[o1];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// The angle-lane sweep: a work-group holds every angle of one sweep direction
// for a segment of cells, lane a <-> angle a of the direction (m = a for
// mu < 0, N/2 + a for mu > 0) and chunk c of the segment (thread c * N/2 + a),
// so a load of psi_{k-1/2} or a store of psi_{k+1/2} and of the outgoing
// fluxes covers consecutive angles of one cell (contiguous in memory).  The
// chunk maps are scanned across the chunks of each angle in LDS; the
// segments' maps across the mesh by k_si_enter (one work-group per angle
// pair); the scalar-flux contribution of a cell sums over the direction's
// angles across the lanes of its chunk group in a fixed order, so the two
// directions leave two partial sums per cell (k_si_reduce adds them).
// ---------------------------------------------------------------------------

// Angle m, direction and position of this thread (threads past the last full
// chunk group idle).
struct LaneMap {
  int NA, C, a, c;
  bool active;
  __device__ __forceinline__ LaneMap(int N) {
    NA = N / 2;
    C = (int)blockDim.x / NA;
    a = (int)threadIdx.x % NA;
    c = (int)threadIdx.x / NA;
    active = c < C;
  }
};

// Chunk at sweep position q of C in a segment [lo, hi): cells [jb, je).
__device__ __forceinline__ void lane_chunk(int lo, int hi, int C, int q, bool pos, int *jb,
                                           int *je) {
  const int n = hi - lo;
  const int k = pos ? q : C - 1 - q;   // chunk index in mesh order
  *jb = lo + (int)(((long long)n * k) / C);
  *je = lo + (int)(((long long)n * (k + 1)) / C);
}

// A chunk swept cell by cell with the loads of the next cell issued before
// the current cell's arithmetic, and the region's data (its 4x4 A_m^{-1},
// dx, sigma_s, Q) kept in registers while the cells stay in one region
// (regions are contiguous cell ranges: the sweep steps into the neighbouring
// region at its edge).  The per-cell arithmetic is cell_solve's.
struct LaneRegion {
  RegionDev g;
  double Ai[16];
  int r;
};

__device__ __forceinline__ void lane_region(const SiArgs &a, int r, int m, LaneRegion &lr) {
  lr.r = r;
  lr.g = a.regions[r];
  const double2 *p = reinterpret_cast<const double2 *>(a.ainv + ((size_t)r * a.N + m) * 16);
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const double2 v = p[i];
    lr.Ai[2 * i] = v.x;
    lr.Ai[2 * i + 1] = v.y;
  }
}

struct LaneIn {
  double2 f01, f23, ps;   // phi_old (4) and psi_{k-1/2} of the cell and angle
};

__device__ __forceinline__ LaneIn lane_in(const double *phi_old, const double *psi_prev, int j,
                                          int m, int K) {
  LaneIn v;
  v.f01 = *reinterpret_cast<const double2 *>(phi_old + (size_t)j * 4);
  v.f23 = *reinterpret_cast<const double2 *>(phi_old + (size_t)j * 4 + 2);
  v.ps = *reinterpret_cast<const double2 *>(psi_prev + (size_t)j * K + 2 * m);
  return v;
}

__device__ __forceinline__ CellSolve lane_solve(const SiArgs &a, const LaneRegion &lr,
                                                const LaneIn &v, bool pos, double amu) {
  const RegionDev &g = lr.g;
  const double po[4] = {v.f01.x, v.f01.y, v.f23.x, v.f23.y};
  double b[4];
  const double qs = g.dx / 4.0;
  for (int c = 0; c < 4; ++c) b[c] = qs * (g.sigs * po[c] + g.q);
  b[0] += a.a * g.dx / 2.0 * v.ps.x;
  b[1] += a.a * g.dx / 2.0 * v.ps.y;
  CellSolve s;
  const int in0 = pos ? 0 : 1, in1 = pos ? 2 : 3;
  const double *Ai = lr.Ai;
  for (int i = 0; i < 4; ++i) {
    s.y[i] = Ai[i * 4 + 0] * b[0] + Ai[i * 4 + 1] * b[1] + Ai[i * 4 + 2] * b[2] + Ai[i * 4 + 3] * b[3];
    s.c0[i] = amu * Ai[i * 4 + in0];
    s.c1[i] = amu * Ai[i * 4 + in1];
  }
  return s;
}

// The region of cell j, stepping from the cached one (sweep direction dir).
__device__ __forceinline__ void lane_track(const SiArgs &a, int j, int m, LaneRegion &lr) {
  if (j >= lr.g.j0 && j < lr.g.j0 + lr.g.nc) return;
  int r = lr.r;
  do {
    r += j >= lr.g.j0 + lr.g.nc ? 1 : -1;
    lane_region(a, r, m, lr);
  } while (j < lr.g.j0 || j >= lr.g.j0 + lr.g.nc);
}

// Map of the chunk [jb, je) in sweep order (as chunk_map).
__device__ Affine lane_chunk_map(const SiArgs &a, const double *phi_old, const double *psi_prev,
                                 int jb, int je, int m, bool pos) {
  const double amu = fabs(a.mu[m]);
  const int o0 = pos ? 1 : 0, o1 = pos ? 3 : 2, K = 2 * a.N, n = je - jb, dir = pos ? 1 : -1;
  Affine f = {1.0, 0.0, 0.0, 1.0, 0.0, 0.0};
  if (n <= 0) return f;
  int j = pos ? jb : je - 1;
  LaneRegion lr;
  lane_region(a, a.cell_region[j], m, lr);
  LaneIn cur = lane_in(phi_old, psi_prev, j, m, K);
  for (int q = 0; q < n; ++q) {
    LaneIn nxt = cur;
    if (q + 1 < n) nxt = lane_in(phi_old, psi_prev, j + dir, m, K);
    lane_track(a, j, m, lr);
    const CellSolve cs = lane_solve(a, lr, cur, pos, amu);
    const Affine g = {cs.c0[o0], cs.c1[o0], cs.c0[o1], cs.c1[o1], cs.y[o0], cs.y[o1]};
    f = compose(g, f);
    cur = nxt;
    j += dir;
  }
  return f;
}

// Segment maps of both directions: grid (nseg, 2), blockIdx.y = pass.
__global__ __launch_bounds__(256) void k_si_smaps(SiArgs a, int node, int cbase) {
  __shared__ Affine s_map[256];
  const StepCtl c = *a.ctl;
  if (c.stalled || c.status != kRunning) return;
  const int l = cbase + node;
  const double *phi_old = ((l - 1) & 1) ? a.phi1 : a.phi0;
  const double *psi_prev = c.step_parity ? a.psi1 : a.psi0;
  const int s = blockIdx.x, pass = blockIdx.y, S = a.nseg;
  const bool pos = pass_positive(a, pass);
  const LaneMap lm(a.N);
  const int lo = seg_edge(s, a.J, S), hi = seg_edge(s + 1, a.J, S);
  if (lm.active) {
    const int m = pos ? lm.NA + lm.a : lm.a;
    int jb, je;
    lane_chunk(lo, hi, lm.C, lm.c, pos, &jb, &je);
    const Affine f = lane_chunk_map(a, phi_old, psi_prev, jb, je, m, pos);
    s_map[threadIdx.x] = f;
    a.chmap[((size_t)pass * S + s) * blockDim.x + threadIdx.x] = f;   // (for k_si_lsweep)
  }
  __syncthreads();
  // the segment's map: the chunks composed in sweep order (one thread per angle)
  if (lm.active && lm.c == 0) {
    Affine f = s_map[lm.a];
    for (int q = 1; q < lm.C; ++q) f = compose(s_map[q * lm.NA + lm.a], f);
    a.segmap[((size_t)pass * S + s) * lm.NA + lm.a] = f;
  }
}

// The flux entering every segment, both directions, for angle pair p =
// blockIdx.x (mu < 0 angle p, mu > 0 angle N-1-p): a scan of the segment maps
// in sweep order (each thread composes a run of consecutive segments, a
// work-group scan joins the runs), applied to the flux entering the mesh.
__global__ __launch_bounds__(256) void k_si_enter(SiArgs a, int node, int cbase) {
  __shared__ Affine s_map[256];
  __shared__ double s_x[2];
  const StepCtl c = *a.ctl;
  if (c.stalled || c.status != kRunning) return;
  const int l = cbase + node;
  const int par = (l - 1) & 1;
  const double *lag_in = a.lag + (size_t)par * a.N;
  double *lag_out = a.lag + (size_t)(l & 1) * a.N;
  const double *ghosts = a.out0;   // ghost rows are identical in both buffers
  const int N = a.N, J = a.J, K = 2 * N, NA = N / 2, S = a.nseg;
  const int p = blockIdx.x;
  const int T = (S + (int)blockDim.x - 1) / (int)blockDim.x;   // segments per thread
  const int q0 = (int)threadIdx.x * T;
  double exit0 = 0.0, exit1 = 0.0;   // pass 0's flux leaving the mesh
  for (int pass = 0; pass < 2; ++pass) {
    const bool pos = pass_positive(a, pass);
    const int m = pos ? N - 1 - p : p, ai = pos ? m - NA : m;
    const Affine *maps = a.segmap + (size_t)pass * S * NA + ai;
    // this thread's run: sweep positions q0 .. q0+T-1 (segment q for mu > 0,
    // S-1-q for mu < 0)
    Affine f = {1.0, 0.0, 0.0, 1.0, 0.0, 0.0};
    for (int q = q0; q < min(q0 + T, S); ++q) f = compose(maps[(size_t)(pos ? q : S - 1 - q) * NA], f);
    scan_maps(f, threadIdx.x, s_map);   // inclusive, in thread order = sweep order
    if (threadIdx.x == 0) {
      double x0 = 0.0, x1 = 0.0;
      if (pos) {
        if (pass == 1 && a.bcl == kBcReflect) { x0 = exit0; x1 = exit1; }
        else if (a.bcl == kBcIncident) { x0 = ghosts[2 * m]; x1 = ghosts[2 * m + 1]; }
      } else {
        if (a.bcr == kBcReflect) {
          if (pass == 1) { x0 = exit0; x1 = exit1; }
          else { x0 = lag_in[2 * p]; x1 = lag_in[2 * p + 1]; }   // both edges reflect
        } else if (a.bcr == kBcIncident) {
          const double *gr = ghosts + (size_t)(J + 1) * K;
          x0 = gr[2 * m];
          x1 = gr[2 * m + 1];
        }
      }
      s_x[0] = x0;
      s_x[1] = x1;
    }
    __syncthreads();
    double x0 = s_x[0], x1 = s_x[1];
    if (threadIdx.x > 0) apply(s_map[threadIdx.x - 1], x0, x1);
    for (int q = q0; q < min(q0 + T, S); ++q) {
      a.segin[((size_t)pass * S + (pos ? q : S - 1 - q)) * NA + ai] = make_double2(x0, x1);
      apply(maps[(size_t)(pos ? q : S - 1 - q) * NA], x0, x1);
    }
    __syncthreads();
    if (threadIdx.x == blockDim.x - 1) {   // the whole mesh's map, applied: the leaving flux
      double y0 = s_x[0], y1 = s_x[1];
      apply(s_map[blockDim.x - 1], y0, y1);
      s_x[0] = y0;
      s_x[1] = y1;
    }
    __syncthreads();
    if (pass == 0) {
      exit0 = s_x[0];
      exit1 = s_x[1];
    } else if (threadIdx.x == 0 && a.bcl == kBcReflect && a.bcr == kBcReflect) {
      // mu > 0 was swept second: its leaving flux at x = X is the next
      // iteration's entering flux of the mirror angle
      lag_out[2 * p] = s_x[0];
      lag_out[2 * p + 1] = s_x[1];
    }
    __syncthreads();
  }
}

// Sum over the NA lanes of a chunk group (NA a power of two <= 64, the group
// contiguous and aligned within a wave): within 16-lane rows by DPP moves
// (pairs, quads, half rows, rows), across rows by lane exchange; each step
// adds a partner's value, so every lane of the group ends with the same sum.
__device__ __forceinline__ double group_sum(double v, int NA) {
  if (NA >= 2) v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]
  if (NA >= 4) v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]
  if (NA >= 8) v += dpp_f64<0x141>(v);   // row_half_mirror
  if (NA >= 16) v += dpp_f64<0x140>(v);  // row_mirror
  if (NA >= 32) v += __shfl_xor(v, 16, 64);
  if (NA >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

// The sweep: grid (nseg, 2), blockIdx.y = pass.  Every thread takes its
// chunk map (formed by k_si_smaps), the flux entering its chunk follows from
// the segment's entering flux through the chunks before it, and the chunk is
// swept from it, writing psi_{k+1/2}, the outgoing fluxes and the
// direction's scalar-flux contribution of every cell.
__global__ __launch_bounds__(256) void k_si_lsweep(SiArgs a, int node, int cbase) {
  __shared__ Affine s_map[256];
  const StepCtl c = *a.ctl;
  if (c.stalled || c.status != kRunning) return;
  const int l = cbase + node;
  const int par = (l - 1) & 1;
  const int parity = c.step_parity;
  const double *phi_old = par ? a.phi1 : a.phi0;
  double *out_dst = par ? a.out0 : a.out1;
  const double *psi_prev = parity ? a.psi1 : a.psi0;
  double *psi_next = parity ? a.psi0 : a.psi1;
  const int N = a.N, J = a.J, K = 2 * N, S = a.nseg;
  const int s = blockIdx.x, pass = blockIdx.y;
  const bool pos = pass_positive(a, pass);
  const LaneMap lm(N);
  const int lo = seg_edge(s, J, S), hi = seg_edge(s + 1, J, S);
  const int m = pos ? lm.NA + lm.a : lm.a;
  const double amu = fabs(a.mu[m]), wm = a.w[m];
  const int o0 = pos ? 1 : 0, o1 = pos ? 3 : 2;
  int jb = lo, je = lo;
  if (lm.active) {
    lane_chunk(lo, hi, lm.C, lm.c, pos, &jb, &je);
    s_map[threadIdx.x] = a.chmap[((size_t)pass * S + s) * blockDim.x + threadIdx.x];
  }
  __syncthreads();
  // the flux entering this chunk: the segment's entering flux through the
  // chunks before it in sweep order
  double x0 = 0.0, x1 = 0.0;
  if (lm.active) {
    const double2 xin = a.segin[((size_t)pass * S + s) * lm.NA + lm.a];
    x0 = xin.x;
    x1 = xin.y;
    for (int q = 0; q < lm.c; ++q) apply(s_map[q * lm.NA + lm.a], x0, x1);
  }
  double *contrib = a.contrib + (size_t)pass * J * 4;
  // (the lanes of a chunk group sweep the same cells in step: equal chunk
  // lengths within the group; groups whose chunk is shorter idle at the end)
  const int n = je - jb, dir = pos ? 1 : -1;
  const int nmax = (hi - lo + lm.C - 1) / max(lm.C, 1) + 1;
  LaneRegion lr;
  LaneIn cur{};
  if (lm.active && n > 0) {
    const int j0 = pos ? jb : je - 1;
    lane_region(a, a.cell_region[j0], m, lr);
    cur = lane_in(phi_old, psi_prev, j0, m, K);
  }
  for (int q = 0; q < nmax; ++q) {
    const bool live = lm.active && q < n;
    double x[4] = {0.0, 0.0, 0.0, 0.0};
    int j = 0;
    if (live) {
      j = pos ? jb + q : je - 1 - q;
      LaneIn nxt = cur;
      if (q + 1 < n) nxt = lane_in(phi_old, psi_prev, j + dir, m, K);
      lane_track(a, j, m, lr);
      const CellSolve cs = lane_solve(a, lr, cur, pos, amu);
      cur = nxt;
      for (int i = 0; i < 4; ++i) x[i] = cs.y[i] + cs.c0[i] * x0 + cs.c1[i] * x1;
      *reinterpret_cast<double2 *>(psi_next + (size_t)j * K + 2 * m) = make_double2(x[2], x[3]);
      *reinterpret_cast<double2 *>(out_dst + (size_t)(j + 1) * K + 2 * m) =
          make_double2(x[o0], x[o1]);
      x0 = x[o0];
      x1 = x[o1];
    }
    // the cell's contribution summed over the group's angles (every lane of
    // the group is live or idle together)
    double sc[4];
    for (int i = 0; i < 4; ++i) sc[i] = group_sum(wm * x[i], lm.NA);
    if (live && lm.a == 0)
      *reinterpret_cast<double4 *>(contrib + (size_t)j * 4) = make_double4(sc[0], sc[1], sc[2], sc[3]);
  }
}

// phi^(l) = sum over the angle pairs' contributions (fixed order), and each
// block's residual record.
__global__ __launch_bounds__(256) void k_si_reduce(SiArgs a, int node, int cb) {
  const StepCtl c = *a.ctl;
  if (c.stalled || c.status != kRunning) return;
  const int l = cb + node;
  const int par = (l - 1) & 1;
  const double *phi_old = par ? a.phi1 : a.phi0;
  double *phi_new = par ? a.phi0 : a.phi1;
  const int J = a.J;
  double d = 0.0, f = 0.0;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < J * 4) {
    double s = 0.0;
    for (int p = 0; p < a.ncontrib; ++p) s += a.contrib[(size_t)p * J * 4 + idx];
    phi_new[idx] = s;
    d = isfinite(s) ? fabs(s - phi_old[idx]) : __builtin_nan("");
    f = fabs(s);
  }
  __shared__ double sd[4], sf[4];
  d = wave_nan_max(d);
  f = wave_max(f);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) { sd[wave] = d; sf[wave] = f; }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    for (int w = 1; w < nw; ++w) {
      d = nan_max(d, sd[w]);
      f = fmax(f, sf[w]);
    }
    reinterpret_cast<double2 *>(a.partial)[(size_t)(l % 3) * a.nparts + blockIdx.x] =
        make_double2(d, f);
  }
}

// Stopping decision for iterate l (one work-group).
__global__ __launch_bounds__(256) void k_si_decide(SiArgs a, int node, int cb) {
  __shared__ double red[2], scratch[2 * 4];
  const StepCtl c = *a.ctl;
  if (c.stalled || c.status != kRunning) return;
  const int l = cb + node;
  const double2 *recs = reinterpret_cast<const double2 *>(a.partial) + (size_t)(l % 3) * a.nparts;
  RecRegs r;
  rec_issue(r, recs, a.nparts);
  rec_finish(r, recs, a.nparts, red, scratch);
  if (threadIdx.x != 0) return;
  double e;
  const int dn = stop_rule(l, red[0], red[1], 0, c.e_prev, 1, a.tol, a.strict, a.max_iters, &e);
  StepCtl *ct = a.ctl;
  if (dn != kRunning) {
    ct->accepted = l;
    ct->e_last = e;
    ct->status = dn;
  } else {
    ct->e_prev = e;
  }
}

// Start of a source-iteration step: the previous step's accepted iterate
// moved into buffer own_buf from buffer fin_buf, and the step opened (the first
// thread leaves the fields the other work-groups read here alone).
__global__ void k_si_begin(SiArgs a, int parity) {
  const StepCtl c = *a.ctl;
  if (c.stalled) return;
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    StepCtl *ct = a.ctl;
    ct->total0 = c.total0 + c.fin_accepted;
    ct->status = kRunning;
    ct->step_parity = parity;
    ct->e_last = -1.0;
    ct->e_prev = -1.0;
  }
  if (c.fin_buf == a.own_buf) return;
  const int K = 2 * a.N;
  const size_t nout = (size_t)a.J * K, nphi = (size_t)a.J * 4;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const double *so = a.outb + (size_t)c.fin_buf * a.out_stride;
  const double *sp = a.phib + (size_t)c.fin_buf * a.phi_stride;
  for (size_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nout; i += stride)
    a.out0[K + i] = so[K + i];
  for (size_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nphi; i += stride)
    a.phi0[i] = sp[i];
}

// End of a decided step: the accepted scalar flux to the result buffer (the
// last sweep already wrote psi_{k+1/2}) and the accepted iterate's lagged
// right-edge flux into lag buffer 0.
__global__ void k_si_end(SiArgs a) {
  const StepCtl c = *a.ctl;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    StepCtl *ct = a.ctl;
    ct->fin_accepted = c.accepted;
    ct->fin_status = c.status;
    ct->fin_e = c.e_last;
    ct->fin_e_prev = c.e_prev;
    if (c.status == kConverged || c.status == kIterLimit) ct->fin_buf = a.own_buf + (c.accepted & 1);
  }
  if (c.stalled || c.status == kRunning || c.status == kNonFinite) return;
  if ((c.accepted & 1) && blockIdx.x == 0)   // the accepted iterate's lag into buffer 0
    for (int i = threadIdx.x; i < a.N; i += blockDim.x) a.lag[i] = a.lag[a.N + i];
  const double *src = (c.accepted & 1) ? a.phi1 : a.phi0;
  const int n = a.J * 4;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    a.phi_res[i] = src[i];
}

}  // namespace ocik
