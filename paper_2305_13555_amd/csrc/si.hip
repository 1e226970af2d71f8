// Source iteration (Sec. "Source Iteration (SI)"): with the scalar flux of
// the previous iteration, every angle is swept through the mesh and each cell
// solves its 4x4 system A^+ x = b^+ (mu > 0) or A^- x = b^- (mu < 0).
//
// On the GPU a sweep is parallel over angles (one work-group per mirror pair
// m, N-1-m) and over cells by a scan: with the lagged scalar flux fixed, the
// map from the flux entering a cell (levels k and k+1/2) to the flux leaving
// it is affine, x_out = T x_in + t, with T = |mu| (A^{-1})[out rows, in rows]
// and t = (A^{-1} b)[out rows].  Each thread composes the maps of a chunk of
// consecutive cells, a work-group scan of the chunk maps gives every chunk
// its entering flux, and each thread re-sweeps its chunk.  The result is the
// sequential sweep up to rounding.
//
// Reflecting edges: the pair is swept in the order that makes the reflection
// exact within the iteration (mu < 0 first when the left edge reflects, mu > 0
// first when only the right edge reflects); with both edges reflecting the
// right edge uses the previous iteration's outgoing flux.
#include "oci_kernels.h"

namespace ocik {


// A^{-1} for every (region, angle): Gauss-Jordan with partial pivoting on the
// unified 4x4 A_m (diagonal (|mu| + dx Sigma)/2, off-diagonal +-mu/2 signed,
// time terms dx/(2 v dt), dx/(v dt)).
__global__ void k_si_invert(const RegionDev *regions, const double *mu, int N, int R, double a,
                            double *ainv) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= R * N) return;
  const int r = idx / N, m = idx % N;
  const RegionDev g = regions[r];
  const double mm = mu[m];
  const double d = (fabs(mm) + g.dx * g.sig) / 2.0, h = mm / 2.0, t = g.dx * a;
  double A[4][8] = {{d, h, t / 2.0, 0.0, 1, 0, 0, 0},
                    {-h, d, 0.0, t / 2.0, 0, 1, 0, 0},
                    {-t, 0.0, t + d, h, 0, 0, 1, 0},
                    {0.0, -t, -h, t + d, 0, 0, 0, 1}};
  for (int k = 0; k < 4; ++k) {
    int p = k;
    for (int i = k + 1; i < 4; ++i)
      if (fabs(A[i][k]) > fabs(A[p][k])) p = i;
    if (p != k)
      for (int j = 0; j < 8; ++j) { const double tmp = A[k][j]; A[k][j] = A[p][j]; A[p][j] = tmp; }
    const double piv = A[k][k];
    for (int j = 0; j < 8; ++j) A[k][j] /= piv;
    for (int i = 0; i < 4; ++i) {
      if (i == k) continue;
      const double l = A[i][k];
      for (int j = 0; j < 8; ++j) A[i][j] -= l * A[k][j];
    }
  }
  double *o = ainv + (size_t)idx * 16;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) o[i * 4 + j] = A[i][4 + j];
}

struct Affine {   // x -> M x + v
  double m00, m01, m10, m11, v0, v1;
};

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

// Iteration l = cb + node: sweep every angle pair with the scalar flux of
// iterate l-1.
__global__ __launch_bounds__(1024) void k_si_sweep(SiArgs a, int node, int cbase) {
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
  const int N = a.N, J = a.J, K = 2 * N;
  const int p = blockIdx.x;
  const int m_neg = p, m_pos = N - 1 - p;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int C = (J + nt - 1) / nt;
  const int jb = min(J, tid * C), je = min(J, (tid + 1) * C);

  __shared__ Affine s_map[1024];
  __shared__ double s_exit[2];

  const bool pos_first = (a.bcr == kBcReflect && a.bcl != kBcReflect);
  double *contrib = a.contrib + (size_t)p * J * 4;
  for (int pass = 0; pass < 2; ++pass) {
    const bool pos = pos_first ? (pass == 0) : (pass == 1);
    const int m = pos ? m_pos : m_neg;
    const double mu = a.mu[m], amu = fabs(mu), wm = a.w[m];
    // flux entering the domain for this direction
    double xb0 = 0.0, xb1 = 0.0;
    if (pos) {
      if (pass == 1 && a.bcl == kBcReflect) { xb0 = s_exit[0]; xb1 = s_exit[1]; }
      else if (a.bcl == kBcIncident) { xb0 = ghosts[2 * m]; xb1 = ghosts[2 * m + 1]; }
    } else {
      if (a.bcr == kBcReflect) {
        if (pass == 1) { xb0 = s_exit[0]; xb1 = s_exit[1]; }
        else { xb0 = a.lag[2 * p]; xb1 = a.lag[2 * p + 1]; }   // both edges reflect
      } else if (a.bcr == kBcIncident) {
        const double *gr = ghosts + (size_t)(J + 1) * K;
        xb0 = gr[2 * m];
        xb1 = gr[2 * m + 1];
      }
    }
    const int o0 = pos ? 1 : 0, o1 = pos ? 3 : 2;
    // phase 1: compose this thread's chunk in sweep order
    Affine f = {1.0, 0.0, 0.0, 1.0, 0.0, 0.0};
    for (int q = 0; q < je - jb; ++q) {
      const int j = pos ? jb + q : je - 1 - q;
      const CellSolve s = cell_solve(a, phi_old, psi_prev, j, m, pos, amu);
      const Affine g = {s.c0[o0], s.c1[o0], s.c0[o1], s.c1[o1], s.y[o0], s.y[o1]};
      f = compose(g, f);
    }
    // phase 2: inclusive scan over threads in sweep order
    const int spos = pos ? tid : nt - 1 - tid;
    s_map[spos] = f;
    __syncthreads();
    for (int off = 1; off < nt; off <<= 1) {
      Affine mine = s_map[spos];
      Affine earlier = {1.0, 0.0, 0.0, 1.0, 0.0, 0.0};
      if (spos >= off) earlier = s_map[spos - off];
      __syncthreads();
      if (spos >= off) s_map[spos] = compose(mine, earlier);
      __syncthreads();
    }
    double x0 = xb0, x1 = xb1;
    if (spos > 0) {
      const Affine e = s_map[spos - 1];
      x0 = e.m00 * xb0 + e.m01 * xb1 + e.v0;
      x1 = e.m10 * xb0 + e.m11 * xb1 + e.v1;
    }
    // phase 3: re-sweep the chunk from its entering flux
    for (int q = 0; q < je - jb; ++q) {
      const int j = pos ? jb + q : je - 1 - q;
      const CellSolve s = cell_solve(a, phi_old, psi_prev, j, m, pos, amu);
      double x[4];
      for (int i = 0; i < 4; ++i) x[i] = s.y[i] + s.c0[i] * x0 + s.c1[i] * x1;
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
    // the thread owning the last cell of the sweep publishes the leaving flux
    const bool owns_last = je > jb && (pos ? je == J : jb == 0);
    if (owns_last) { s_exit[0] = x0; s_exit[1] = x1; }
    __syncthreads();
  }
  if (a.bcl == kBcReflect && a.bcr == kBcReflect && tid == 0) {
    // mu > 0 was swept second: its leaving flux at x = X is next iteration's
    // entering flux of the mirror angle
    a.lag[2 * p] = s_exit[0];
    a.lag[2 * p + 1] = s_exit[1];
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
  const int npairs = a.N / 2;
  const int J = a.J;
  double d = 0.0, f = 0.0;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < J * 4) {
    double s = 0.0;
    for (int p = 0; p < npairs; ++p) s += a.contrib[(size_t)p * J * 4 + idx];
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

// Start of a source-iteration step: the previous step's last iterate moved
// into buffer 0 when it sits in buffer 1, and the step opened (the first
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
  if (!(c.fin_accepted & 1)) return;
  const int K = 2 * a.N;
  const size_t nout = (size_t)a.J * K, nphi = (size_t)a.J * 4;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nout; i += stride)
    a.out0[K + i] = a.out1[K + i];
  for (size_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nphi; i += stride)
    a.phi0[i] = a.phi1[i];
}

// End of a decided step: the accepted scalar flux to the result buffer (the
// last sweep already wrote psi_{k+1/2}).
__global__ void k_si_end(SiArgs a) {
  const StepCtl c = *a.ctl;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    StepCtl *ct = a.ctl;
    ct->fin_accepted = c.accepted;
    ct->fin_status = c.status;
    ct->fin_e = c.e_last;
  }
  if (c.stalled || c.status == kRunning || c.status == kNonFinite) return;
  const double *src = (c.accepted & 1) ? a.phi1 : a.phi0;
  const int n = a.J * 4;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    a.phi_res[i] = src[i];
}

}  // namespace ocik
