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

// One work-group per region: the operator rows op [2N+4+2N][4N+1] (outgoing
// fluxes, scalar flux, time-edge values; columns: incident 2N, time edge 2N,
// source) from the A_m^{-1} (ainv [R][N][16]), and the scalar-flux rows of
// its incident columns once more, plain: phig [R][4][2N].  Dynamic LDS:
// (32N + 4) doubles.  A singular or non-finite 4x4 system sets *bad.
__global__ __launch_bounds__(256) void k_cell_operator(const RegionDev *regions,
                                                        const double *mu, const double *w,
                                                        const double *ainv, int N, double a,
                                                        double *op_all, double *phig, int *bad) {
  extern __shared__ double sh[];
  __shared__ double Ks[16], Kinv[16];
  const int r = blockIdx.x, tid = threadIdx.x;
  const int n = 4 * N, nr = n + 1, rows = 4 * N + 4;
  double *Ai = sh;            // [N][4][4]: A_m^{-1}
  double *Ph = sh + 16 * N;   // [4][nr]: Phi
  const RegionDev g = regions[r];
  const double s = g.dx * g.sigs / 4.0, th = g.dx * a / 2.0, qq = g.dx * g.q / 4.0;
  for (int i = tid; i < 16 * N; i += blockDim.x) Ai[i] = ainv[(size_t)r * N * 16 + i];
  __syncthreads();
  // K = I - s sum_m w_m A_m^{-1}
  if (tid < 16) {
    double acc = 0.0;
    for (int m = 0; m < N; ++m) acc += w[m] * Ai[m * 16 + tid];
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
    if (!ok) *bad = 1;
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
      const double f = w[m] * (inc ? fabs(mu[m]) : th);
#pragma unroll
      for (int c = 0; c < 4; ++c) v[c] = f * Ai[m * 16 + c * 4 + cc];
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        double acc = 0.0;
        for (int m = 0; m < N; ++m) {
          const double *A = Ai + m * 16 + c * 4;
          acc += w[m] * (A[0] + A[1] + A[2] + A[3]);
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
  for (int i = tid; i < 4 * 2 * N; i += blockDim.x)
    phig[(size_t)r * 8 * N + i] = Ph[(i / (2 * N)) * nr + i % (2 * N)];
  // Y rows: angle m, corner c: (A_m^{-1} [B|T|q])[(m,c), col] + s (A_m^{-1} Phi)[c, col]
  double *op = op_all + (size_t)r * rows * nr;
  for (int idx = tid; idx < rows * nr; idx += blockDim.x) {
    const int row = idx / nr, col = idx - row * nr;
    double val;
    if (row >= 2 * N && row < 2 * N + 4) {
      val = Ph[(row - 2 * N) * nr + col];
    } else {
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
        if ((col >> 1) == m) own = fabs(mu[m]) * A[entering_corner(m, N, col & 1)];
      } else if (col < 4 * N) {
        const int p = col - 2 * N;
        if ((p >> 1) == m) own = th * A[p & 1];
      } else {
        own = qq * (A[0] + A[1] + A[2] + A[3]);
      }
      val = own + s * (A[0] * Ph[col] + A[1] * Ph[nr + col] + A[2] * Ph[2 * nr + col] +
                       A[3] * Ph[3 * nr + col]);
    }
    op[idx] = val;
  }
}

// Pack a rows x K block of the operator (first row row0, first column col0)
// into MFMA fragment order: frag[(rt*KS + ks)*64 + lane] =
// A[rt*16 + lane%16][k] with k = ks*4 + lane/16, or with kmajor
// k = (lane/16)*KS + ks (zero beyond `rows`), KS = K/4, and the constant
// column into cvec[rt*16 + i] (zero-padded to Mt*16).
__global__ void k_pack(int N, const double *op_all, int row0, int rows, int col0, int K,
                       int Mt, double *frag_all, size_t frag_stride, double *cvec_all,
                       size_t cvec_stride, int kmajor) {
  const int r = blockIdx.x;
  const int nr = 4 * N + 1;
  const int oprows = 4 * N + 4;
  const double *op = op_all + (size_t)r * oprows * nr;
  double *frag = frag_all + (size_t)r * frag_stride;
  const int KS = K / 4;
  const int total = Mt * KS * 64;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int lane = idx & 63;
    const int blk = idx >> 6;
    const int rt = blk / KS, ks = blk % KS;
    const int row = rt * 16 + (lane & 15);
    const int col = kmajor ? (lane >> 4) * KS + ks : ks * 4 + (lane >> 4);
    frag[idx] = row < rows ? op[(size_t)(row0 + row) * nr + col0 + col] : 0.0;
  }
  if (cvec_all) {
    double *cv = cvec_all + (size_t)r * cvec_stride;
    for (int i = threadIdx.x; i < Mt * 16; i += blockDim.x)
      cv[i] = i < rows ? op[(size_t)(row0 + i) * nr + 4 * N] : 0.0;
  }
}


// Coefficients of the structured OCI apply for every (region, angle), from
// A_m^{-1}: the outgoing corner rows o_t (levels t = k, k+1/2) act on the
// scattering source s phi (s = dx Sigma_s / 4), the entering fluxes |mu| inc
// (entering-corner columns in_t), and give the step constant from the source
// (dx Q / 4 in every row) and the time edge (dx / (2 v dt) psi_{k-1/2} in the
// two level-k rows).  Layout: pairs of coefficients, pair-major: values 2p
// and 2p+1 of (region r, angle m) at coef[((r * kCoef/2 + p) * N + m) * 2 + 0/1],
// so that a thread loads two with one instruction and the threads of a
// work-group (consecutive angles) read consecutive addresses.  Use:
// oci_step.hip, "The structured apply".
__global__ void k_out_coef(const RegionDev *regions, const double *mu, const double *ainv, int N,
                           int R, double a, double *coef) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= R * N) return;
  const int r = idx / N, m = idx % N;
  const RegionDev g = regions[r];
  const bool pos = 2 * m >= N;   // mu > 0: outgoing at the right corner
  const int o[2] = {pos ? 1 : 0, pos ? 3 : 2};
  const int in0 = pos ? 0 : 1, in1 = pos ? 2 : 3;
  const double s = g.dx * g.sigs / 4.0, amu = fabs(mu[m]);
  const double qq = g.dx * g.q / 4.0, ts = a * g.dx / 2.0;
  const double *Ai = ainv + (size_t)idx * 16;
  double cf[kCoef];
  for (int t = 0; t < 2; ++t) {
    const double *row = Ai + o[t] * 4;
    for (int c = 0; c < 4; ++c) cf[6 * t + c] = s * row[c];
    cf[6 * t + 4] = amu * row[in0];
    cf[6 * t + 5] = amu * row[in1];
    cf[12 + 3 * t] = qq * (row[0] + row[1] + row[2] + row[3]);
    cf[13 + 3 * t] = ts * row[0];
    cf[14 + 3 * t] = ts * row[1];
  }
  // psi_{k+1/2} at L and R: rows 2 and 3
  for (int u = 0; u < 2; ++u) {
    const double *row = Ai + (2 + u) * 4;
    for (int c = 0; c < 4; ++c) cf[18 + 9 * u + c] = s * row[c];
    cf[22 + 9 * u] = ts * row[0];
    cf[23 + 9 * u] = ts * row[1];
    cf[24 + 9 * u] = amu * row[in0];
    cf[25 + 9 * u] = amu * row[in1];
    cf[26 + 9 * u] = qq * (row[0] + row[1] + row[2] + row[3]);
  }
  for (int k = 0; k < kCoef; ++k) coef[(((size_t)r * (kCoef / 2) + k / 2) * N + m) * 2 + (k & 1)] = cf[k];
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
