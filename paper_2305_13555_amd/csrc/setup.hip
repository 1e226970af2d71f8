// Setup kernels: the per-region cell operator and its packed forms applied
// on the hot path.
//
// The cell system of one-cell inversion (Sec. "One-Cell Inversion (OCI)") is
// (A - S) Psi = c with A = blockdiag(A_m), A_m the 4x4 matrix printed for
// mu > 0 (A^+) and mu < 0 (A^-) in the SI subsection, and S the scattering
// matrix with entries (dx Sigma_s / 4) w_n coupling equal components of all
// angles.  Both signs of A_m are one formula: diagonal (|mu| + dx Sigma)/2,
// off-diagonal +-mu/2 with the signed mu, and the time terms dx/(2 v dt),
// dx/(v dt).  All cells of a region share A - S.
//
// c enters through three sets of columns: the incident fluxes (coefficient
// |mu_m| in the c^+ / c^- rows that carry them), the previous time edge
// psi_{k-1/2} (coefficient dx/(2 v dt) in the two time-average rows) and the
// source (dx Q / 4 in every row).  Setup solves (A - S) Y = [B | T | q] once
// per region and keeps only the rows the iteration needs: the outgoing
// fluxes, the scalar flux and the time-edge values.
//
// The paper solves the cell system with a dense direct solver.  Here the
// solve uses its structure: S = s E W with s = dx Sigma_s / 4, (W psi)_c =
// sum_m w_m psi_{m,c} (the scalar flux) and (E phi)_{m,c} = phi_c.  Then
//   Y = A^{-1} [B|T|q] + s A^{-1} E Phi,   Phi = W Y,
//   (I - s sum_m w_m A_m^{-1}) Phi = W A^{-1} [B|T|q],
// a 4x4 system per region (the same solution as the dense solve up to
// rounding, in O(N) work per column instead of O(N^2) per column after an
// O(N^3) factorisation), with the A_m^{-1} of the SI sweep.
#include "oci_kernels.h"

namespace ocik {

// Entering corner of angle m's incident value tl (0: level k, 1: k+1/2),
// and the outgoing corner of its outgoing value tl: mu < 0 (m < N/2) enters
// on the right (corners 1, 3) and leaves on the left (0, 2).
__device__ __forceinline__ int entering_corner(int m, int N, int tl) {
  return m < N / 2 ? (tl == 0 ? 1 : 3) : (tl == 0 ? 0 : 2);
}
__device__ __forceinline__ int outgoing_corner(int m, int N, int tl) {
  return m < N / 2 ? (tl == 0 ? 0 : 2) : (tl == 0 ? 1 : 3);
}

// A_m^{-1} of the unified 4x4 A_m (diagonal (|mu| + dx Sigma)/2,
// off-diagonal +-mu/2 signed, time terms dx/(2 v dt), dx/(v dt)): Gauss-Jordan
// with partial pivoting; out row-major.  Every loop is unrolled and the row
// swap done by selects, so the matrix stays in registers.
__device__ __forceinline__ void invert_cell_matrix(double mm, const RegionDev &g, double a,
                                                   double out[16]) {
  const double d = (fabs(mm) + g.dx * g.sig) / 2.0, h = mm / 2.0, t = g.dx * a;
  double A[4][8] = {{d, h, t / 2.0, 0.0, 1, 0, 0, 0},
                    {-h, d, 0.0, t / 2.0, 0, 1, 0, 0},
                    {-t, 0.0, t + d, h, 0, 0, 1, 0},
                    {0.0, -t, -h, t + d, 0, 0, 0, 1}};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int p = k;
    double best = fabs(A[k][k]);
#pragma unroll
    for (int i = k + 1; i < 4; ++i)
      if (fabs(A[i][k]) > best) {
        best = fabs(A[i][k]);
        p = i;
      }
#pragma unroll
    for (int i = k + 1; i < 4; ++i)
      if (i == p)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const double tmp = A[k][j];
          A[k][j] = A[i][j];
          A[i][j] = tmp;
        }
    const double piv = A[k][k];
#pragma unroll
    for (int j = 0; j < 8; ++j) A[k][j] /= piv;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (i == k) continue;
      const double l = A[i][k];
#pragma unroll
      for (int j = 0; j < 8; ++j) A[i][j] -= l * A[k][j];
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) out[i * 4 + j] = A[i][4 + j];
}

// Coefficients of the structured OCI apply for one (region r, angle m), from
// Ai = A_m^{-1}: the outgoing corner rows o_t (levels t = k, k+1/2) act on the
// scattering source s phi (s = dx Sigma_s / 4), the entering fluxes |mu| inc
// (entering-corner columns in_t), and give the step constant from the source
// (dx Q / 4 in every row) and the time edge (dx / (2 v dt) psi_{k-1/2} in the
// two level-k rows).  Layout: pairs of coefficients, pair-major: values 2p
// and 2p+1 of (region r, angle m) at coef[((r * kCoef/2 + p) * N + m) * 2 + 0/1],
// so that a thread loads two with one instruction and the threads of a
// work-group (consecutive angles) read consecutive addresses.  Use:
// oci_step.hip, "The structured apply".
__device__ __forceinline__ void write_out_coef(const double Ai[16], const RegionDev &g, double mum,
                                               int r, int m, int N, double a, double *coef) {
  const bool pos = 2 * m >= N;   // mu > 0: outgoing at the right corner
  const int in0 = pos ? 0 : 1, in1 = pos ? 2 : 3;
  const double s = g.dx * g.sigs / 4.0, amu = fabs(mum);
  const double qq = g.dx * g.q / 4.0, ts = a * g.dx / 2.0;
  // outgoing rows (R0: level k, R1: level k+1/2) and the rows 2, 3 of Ai,
  // chosen by selects (Ai stays in registers)
  double R0[4], R1[4], R2[4], R3[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    R2[c] = Ai[8 + c];
    R3[c] = Ai[12 + c];
    R0[c] = pos ? Ai[4 + c] : Ai[c];
    R1[c] = pos ? R3[c] : R2[c];
  }
  auto pick = [](const double *rw, int cs) {
    return cs == 0 ? rw[0] : cs == 1 ? rw[1] : cs == 2 ? rw[2] : rw[3];
  };
  double cf[kCoef];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const double *rw = t == 0 ? R0 : R1;
#pragma unroll
    for (int c = 0; c < 4; ++c) cf[6 * t + c] = s * rw[c];
    cf[6 * t + 4] = amu * pick(rw, in0);
    cf[6 * t + 5] = amu * pick(rw, in1);
    cf[12 + 3 * t] = qq * (rw[0] + rw[1] + rw[2] + rw[3]);
    cf[13 + 3 * t] = ts * rw[0];
    cf[14 + 3 * t] = ts * rw[1];
  }
  // psi_{k+1/2} at L and R: rows 2 and 3
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const double *rw = u == 0 ? R2 : R3;
#pragma unroll
    for (int c = 0; c < 4; ++c) cf[18 + 9 * u + c] = s * rw[c];
    cf[22 + 9 * u] = ts * rw[0];
    cf[23 + 9 * u] = ts * rw[1];
    cf[24 + 9 * u] = amu * pick(rw, in0);
    cf[25 + 9 * u] = amu * pick(rw, in1);
    cf[26 + 9 * u] = qq * (rw[0] + rw[1] + rw[2] + rw[3]);
  }
#pragma unroll
  for (int k = 0; k < kCoef / 2; ++k)
    reinterpret_cast<double2 *>(coef)[((size_t)r * (kCoef / 2) + k) * N + m] =
        make_double2(cf[2 * k], cf[2 * k + 1]);
}

// Every per-region table of the solve in one launch, grid (R, NB) of 256
// threads.  Each work-group of region r forms, in LDS, the A_m^{-1} of all
// angles, K = I - s sum_m w_m A_m^{-1}, K^{-1} and Phi = K^{-1} W A^{-1}
// [B|T|q] (cheap; repeated per work-group so that the NB work-groups of a
// region need no ordering between them).  Work-group (r, 0) writes ainv
// [R][N][16], the structured-apply coefficients and phig [R][4][2N] (the
// scalar-flux rows of the incident columns, plain); the NB work-groups of the
// region share the rest: the operator rows op [R][2N+4+2N][4N+1] (outgoing
// fluxes, scalar flux, time-edge values; columns: incident 2N, time edge 2N,
// source), G = rows [0, 2N+4) x incident columns and P = the same rows x
// time-edge columns in MFMA fragment order, k-major:
// frag[(rt*KS + ks)*64 + lane] = Y[rt*16 + lane%16][(lane/16)*KS + ks],
// KS = N/2, zero beyond row 2N+3 (G once more in FP32 for the mixed-precision
// solve), and the source column p (zero-padded to Mt*16).  A singular or
// non-finite 4x4 system K sets *bad.  Dynamic LDS: (32N + 4) doubles.
__global__ __launch_bounds__(256) void k_region_setup(SetupArgs q) {
  extern __shared__ double sh[];
  __shared__ double Ks[16], Kinv[16];
  const int r = blockIdx.x, y = blockIdx.y, tid = threadIdx.x;
  const int N = q.N, n = 4 * N, nr = n + 1, rows = 4 * N + 4;
  double *Ai = sh;            // [N][4][4]: A_m^{-1}
  double *Ph = sh + 16 * N;   // [4][nr]: Phi
  const RegionDev g = q.regions[r];
  const double s = g.dx * g.sigs / 4.0, th = g.dx * q.a / 2.0, qq = g.dx * g.q / 4.0;
  for (int m = tid; m < N; m += blockDim.x) {
    double A[16];
    invert_cell_matrix(q.mu[m], g, q.a, A);
#pragma unroll
    for (int i = 0; i < 16; ++i) Ai[m * 16 + i] = A[i];
    if (y == 0) {
      double2 *o = reinterpret_cast<double2 *>(q.ainv + ((size_t)r * N + m) * 16);
#pragma unroll
      for (int i = 0; i < 8; ++i) o[i] = make_double2(A[2 * i], A[2 * i + 1]);
      write_out_coef(A, g, q.mu[m], r, m, N, q.a, q.coef);
    }
  }
  __syncthreads();
  // K = I - s sum_m w_m A_m^{-1}
  if (tid < 16) {
    double acc = 0.0;
    for (int m = 0; m < N; ++m) acc += q.w[m] * Ai[m * 16 + tid];
    Ks[tid] = ((tid >> 2) == (tid & 3) ? 1.0 : 0.0) - s * acc;
  }
  __syncthreads();
  if (tid == 0) {   // K^{-1}: Gauss-Jordan with partial pivoting
    double M[4][8];
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        M[i][j] = Ks[i * 4 + j];
        M[i][4 + j] = i == j ? 1.0 : 0.0;
      }
    bool ok = true;
    // (loops unrolled, the row swap by selects: M stays in registers)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      int p = k;
      double best = fabs(M[k][k]);
#pragma unroll
      for (int i = k + 1; i < 4; ++i)
        if (fabs(M[i][k]) > best) {
          best = fabs(M[i][k]);
          p = i;
        }
#pragma unroll
      for (int i = k + 1; i < 4; ++i)
        if (i == p)
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const double tmp = M[k][j];
            M[k][j] = M[i][j];
            M[i][j] = tmp;
          }
      const double piv = M[k][k];
      if (!(fabs(piv) > 0.0) || !isfinite(piv)) ok = false;
#pragma unroll
      for (int j = 0; j < 8; ++j) M[k][j] /= piv;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (i == k) continue;
        const double l = M[i][k];
#pragma unroll
        for (int j = 0; j < 8; ++j) M[i][j] -= l * M[k][j];
      }
    }
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        Kinv[i * 4 + j] = M[i][4 + j];
        if (!isfinite(M[i][4 + j])) ok = false;
      }
    if (!ok && y == 0) *q.bad = 1;
  }
  __syncthreads();
  // Phi[:, col] = K^{-1} (W A^{-1} [B|T|q])[:, col]: an incident or time-edge
  // column has one nonzero (one angle's row), the source column all rows
  for (int col = tid; col < nr; col += blockDim.x) {
    double v[4];
    if (col < 4 * N) {
      const bool inc = col < 2 * N;
      const int p = inc ? col : col - 2 * N, m = p >> 1, tl = p & 1;
      const int cc = inc ? entering_corner(m, N, tl) : tl;   // time edge: level-k row tl
      const double f = q.w[m] * (inc ? fabs(q.mu[m]) : th);
#pragma unroll
      for (int c = 0; c < 4; ++c) v[c] = f * Ai[m * 16 + c * 4 + cc];
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        double acc = 0.0;
        for (int m = 0; m < N; ++m) {
          const double *A = Ai + m * 16 + c * 4;
          acc += q.w[m] * (A[0] + A[1] + A[2] + A[3]);
        }
        v[c] = qq * acc;
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
      Ph[c * nr + col] = Kinv[c * 4 + 0] * v[0] + Kinv[c * 4 + 1] * v[1] +
                         Kinv[c * 4 + 2] * v[2] + Kinv[c * 4 + 3] * v[3];
  }
  __syncthreads();
  if (y == 0)
    for (int i = tid; i < 4 * 2 * N; i += blockDim.x)
      q.phig[(size_t)r * 8 * N + i] = Ph[(i / (2 * N)) * nr + i % (2 * N)];
  // Y rows: angle m, corner c: (A_m^{-1} [B|T|q])[(m,c), col] + s (A_m^{-1} Phi)[c, col]
  auto val = [&](int row, int col) -> double {
    if (row >= 2 * N && row < 2 * N + 4) return Ph[(row - 2 * N) * nr + col];
    int m, c;
    if (row < 2 * N) {
      m = row >> 1;
      c = outgoing_corner(m, N, row & 1);
    } else {
      const int p = row - 2 * N - 4;
      m = p >> 1;
      c = 2 + (p & 1);
    }
    const double *A = Ai + m * 16 + c * 4;   // row c of A_m^{-1}
    double own = 0.0;
    if (col < 2 * N) {
      if ((col >> 1) == m) own = fabs(q.mu[m]) * A[entering_corner(m, N, col & 1)];
    } else if (col < 4 * N) {
      const int p = col - 2 * N;
      if ((p >> 1) == m) own = th * A[p & 1];
    } else {
      own = qq * (A[0] + A[1] + A[2] + A[3]);
    }
    return own + s * (A[0] * Ph[col] + A[1] * Ph[nr + col] + A[2] * Ph[2 * nr + col] +
                      A[3] * Ph[3 * nr + col]);
  };
  const int first = y * blockDim.x + tid, stride = gridDim.y * blockDim.x;
  double *op = q.op + (size_t)r * rows * nr;
  for (int idx = first; idx < rows * nr; idx += stride) {
    const int row = idx / nr;
    op[idx] = val(row, idx - row * nr);
  }
  const int KS = N / 2, total = q.Mt * KS * 64, grows = 2 * N + 4;
  double *fi = q.frag_it + (size_t)r * q.frag_stride;
  double *fp = q.frag_pv + (size_t)r * q.frag_stride;
  float *fi32 = q.frag_it32 ? q.frag_it32 + (size_t)r * q.frag_stride : nullptr;
  for (int idx = first; idx < 2 * total; idx += stride) {
    const bool pv = idx >= total;
    const int e = pv ? idx - total : idx;
    const int lane = e & 63, blk = e >> 6;
    const int rt = blk / KS, ks = blk - rt * KS;
    const int row = rt * 16 + (lane & 15);
    const int col = (lane >> 4) * KS + ks + (pv ? 2 * N : 0);
    const double v = row < grows ? val(row, col) : 0.0;
    if (pv) {
      fp[e] = v;
    } else {
      fi[e] = v;
      if (fi32) fi32[e] = (float)v;
    }
  }
  double *cv = q.c_pv + (size_t)r * q.cvec_stride;
  for (int i = first; i < q.Mt * 16; i += stride) cv[i] = i < grows ? val(i, 4 * N) : 0.0;
}

// Clear z.count ranges of doubles (one launch instead of one fill per range).
__global__ void k_zero(ZeroRanges z) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (int r = 0; r < z.count; ++r) {
    double *p = z.p[r];
    const size_t n = z.n[r];
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0.0;
  }
}

}  // namespace ocik
