// Setup kernels: per-region cell matrix, its LU factorisation, and the packed
// operators applied on the hot path.
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
// per region by LU with partial pivoting (the paper's dense solver, LAPACK
// gesv, hoisted out of the iteration) and keeps only the rows the iteration
// needs: the outgoing fluxes, the scalar flux and the time-edge values.
#include "oci_kernels.h"

namespace ocik {

// One work-group per region: M (n x n, n = 4N) and the right-hand sides
// X (n x (n+1)) into the workspace.
__global__ void k_build_system(const RegionDev *regions, const double *mu, const double *w,
                               int N, double a, double *ws_M, double *ws_X) {
  const int r = blockIdx.x;
  const int n = 4 * N, nr = n + 1;
  const RegionDev g = regions[r];
  double *M = ws_M + (size_t)r * n * n;
  double *X = ws_X + (size_t)r * n * nr;
  const double dx = g.dx;
  const double t = dx * a;               // dx / (v dt)
  const double s = dx * g.sigs / 4.0;    // scattering coefficient
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int row = idx / n, col = idx % n;
    const int m = row >> 2, c = row & 3, mm = col >> 2, cc = col & 3;
    double v = 0.0;
    if (m == mm) {
      const double mum = mu[m];
      const double d = (fabs(mum) + dx * g.sig) / 2.0;
      const double h = mum / 2.0;
      // rows: (k,L) (k,R) (k+1/2,L) (k+1/2,R)
      const double A[4][4] = {{d, h, t / 2.0, 0.0},
                              {-h, d, 0.0, t / 2.0},
                              {-t, 0.0, t + d, h},
                              {0.0, -t, -h, t + d}};
      v = A[c][cc];
    }
    if (c == cc) v -= s * w[mm];
    M[idx] = v;
  }
  for (int idx = threadIdx.x; idx < n * nr; idx += blockDim.x) {
    const int row = idx / nr, col = idx % nr;
    const int m = row >> 2, c = row & 3;
    double v = 0.0;
    if (col < 2 * N) {
      // incident entry 2m'+tl: enters row (m', c_in) with |mu|
      const int mi = col >> 1, tl = col & 1;
      if (mi == m) {
        const int cin = (m < N / 2) ? (tl == 0 ? 1 : 3) : (tl == 0 ? 0 : 2);
        if (c == cin) v = fabs(mu[m]);
      }
    } else if (col < 4 * N) {
      // previous time edge 2m'+side: enters the time-average row of that side
      const int p = col - 2 * N;
      if ((p >> 1) == m && (p & 1) == c) v = t / 2.0;
    } else {
      v = dx * g.q / 4.0;
    }
    X[idx] = v;
  }
}

// The same LU with partial pivoting with the work in LDS, for 4N <= 128.
// Work-group (r, b) holds all of M (n x n) and columns [b*CB, b*CB+CB) of X
// side by side in LDS rows of pitch P (odd, so that column walks spread over
// the banks); every work-group of a region factors M again (cheap next to a
// round trip to memory per pivot) and carries its own block of X along, so
// the right-hand sides are split over several CUs.  The pivot sequence and
// every floating-point operation are those of k_lu_solve: first maximum of
// |column| as pivot, multipliers M[i][k] / M[k][k], rank-one updates, then
// back substitution row by row.  Singular pivots set *bad.
__global__ __launch_bounds__(1024) void k_lu_solve_lds(int N, int CB, int P, const double *ws_M,
                                                       double *ws_X, int *bad) {
  extern __shared__ double A[];
  __shared__ int s_piv;
  __shared__ double s_pv;
  const int r = blockIdx.x, j0 = blockIdx.y * CB;
  const int n = 4 * N, nr = n + 1, Wd = n + CB;
  const int ncol = min(CB, nr - j0);
  const double *M = ws_M + (size_t)r * n * n;
  double *X = ws_X + (size_t)r * n * nr;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  for (int idx = tid; idx < n * Wd; idx += blockDim.x) {
    const int i = idx / Wd, j = idx - i * Wd;
    double v = 0.0;
    if (j < n) v = M[(size_t)i * n + j];
    else if (j - n < ncol) v = X[(size_t)i * nr + j0 + (j - n)];
    A[i * P + j] = v;
  }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (wave == 0) {
      double best = -1.0;
      int bi = n;
      for (int i = k + lane; i < n; i += 64) {
        const double v = fabs(A[i * P + k]);
        if (v > best) { best = v; bi = i; }
      }
      for (int o = 32; o > 0; o >>= 1) {
        const double v2 = __shfl_xor(best, o, 64);
        const int i2 = __shfl_xor(bi, o, 64);
        if (v2 > best || (v2 == best && i2 < bi)) { best = v2; bi = i2; }
      }
      if (lane == 0) {
        s_piv = bi;
        s_pv = best;
      }
    }
    __syncthreads();
    const int p = s_piv;
    if (!(s_pv > 0.0)) {
      if (tid == 0) *bad = 1;
      return;   // uniform: every thread read the same s_pv
    }
    if (p != k) {
      for (int j = k + tid; j < Wd; j += blockDim.x) {
        const double tmp = A[k * P + j];
        A[k * P + j] = A[p * P + j];
        A[p * P + j] = tmp;
      }
      __syncthreads();
    }
    const double piv = A[k * P + k];
    for (int i = k + 1 + tid; i < n; i += blockDim.x) A[i * P + k] = A[i * P + k] / piv;
    __syncthreads();
    for (int i = k + 1 + wave; i < n; i += nw) {
      const double l = A[i * P + k];
      for (int j = k + 1 + lane; j < Wd; j += 64) A[i * P + j] -= l * A[k * P + j];
    }
    __syncthreads();
  }
  for (int k = n - 1; k >= 0; --k) {
    const double piv = A[k * P + k];
    for (int j = tid; j < CB; j += blockDim.x) A[k * P + n + j] /= piv;
    __syncthreads();
    for (int i = wave; i < k; i += nw) {
      const double u = A[i * P + k];
      for (int j = lane; j < CB; j += 64) A[i * P + n + j] -= u * A[k * P + n + j];
    }
    __syncthreads();
  }
  for (int idx = tid; idx < n * ncol; idx += blockDim.x) {
    const int i = idx / ncol, j = idx - i * ncol;
    X[(size_t)i * nr + j0 + j] = A[i * P + n + j];
  }
}

// LU with partial pivoting of M, applied to X at the same time, then back
// substitution: X <- M^{-1} X.  One work-group per region; singular pivots set
// *bad.
__global__ __launch_bounds__(1024) void k_lu_solve(int N, double *ws_M, double *ws_X, int *bad) {
  const int r = blockIdx.x;
  const int n = 4 * N, nr = n + 1;
  double *M = ws_M + (size_t)r * n * n;
  double *X = ws_X + (size_t)r * n * nr;
  __shared__ double s_val[1024];
  __shared__ int s_idx[1024];
  __shared__ double s_l[1024];
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int k = 0; k < n; ++k) {
    // pivot search on column k (first maximum, like LAPACK's idamax)
    double best = -1.0;
    int bi = n;
    for (int i = k + tid; i < n; i += nt) {
      const double v = fabs(M[(size_t)i * n + k]);
      if (v > best) { best = v; bi = i; }
    }
    s_val[tid] = best;
    s_idx[tid] = bi;
    __syncthreads();
    for (int o = nt / 2; o > 0; o >>= 1) {
      if (tid < o) {
        const double v2 = s_val[tid + o];
        const int i2 = s_idx[tid + o];
        if (v2 > s_val[tid] || (v2 == s_val[tid] && i2 < s_idx[tid])) {
          s_val[tid] = v2;
          s_idx[tid] = i2;
        }
      }
      __syncthreads();
    }
    const int p = s_idx[0];
    const double pv = s_val[0];
    if (!(pv > 0.0)) {
      if (tid == 0) *bad = 1;
      return;   // uniform: every thread saw the same s_val[0]
    }
    if (p != k) {
      for (int j = k + tid; j < n; j += nt) {
        const double tmp = M[(size_t)k * n + j];
        M[(size_t)k * n + j] = M[(size_t)p * n + j];
        M[(size_t)p * n + j] = tmp;
      }
      for (int j = tid; j < nr; j += nt) {
        const double tmp = X[(size_t)k * nr + j];
        X[(size_t)k * nr + j] = X[(size_t)p * nr + j];
        X[(size_t)p * nr + j] = tmp;
      }
    }
    __syncthreads();
    const double piv = M[(size_t)k * n + k];
    for (int i = k + 1 + tid; i < n; i += nt) s_l[i - k - 1] = M[(size_t)i * n + k] / piv;
    __syncthreads();
    const int rows = n - k - 1;
    const int wM = n - k - 1;     // columns k+1 .. n-1 of M
    const int wT = wM + nr;       // followed by every column of X
    for (int idx = tid; idx < rows * wT; idx += nt) {
      const int ii = idx / wT, jj = idx % wT;
      const int i = k + 1 + ii;
      const double l = s_l[ii];
      if (jj < wM) {
        const int j = k + 1 + jj;
        M[(size_t)i * n + j] -= l * M[(size_t)k * n + j];
      } else {
        const int j = jj - wM;
        X[(size_t)i * nr + j] -= l * X[(size_t)k * nr + j];
      }
    }
    __syncthreads();
  }
  for (int k = n - 1; k >= 0; --k) {
    const double piv = M[(size_t)k * n + k];
    for (int j = tid; j < nr; j += nt) X[(size_t)k * nr + j] /= piv;
    __syncthreads();
    for (int idx = tid; idx < k * nr; idx += nt) {
      const int i = idx / nr, j = idx % nr;
      X[(size_t)i * nr + j] -= M[(size_t)i * n + k] * X[(size_t)k * nr + j];
    }
    __syncthreads();
  }
}

// Row selection of Y = M^{-1}[B|T|q] into the per-region operator
// op [2N+4+2N][4N+1]: outgoing fluxes, scalar flux (sum_n w_n psi_n),
// time-edge values.
__global__ void k_select_rows(int N, const double *w, const double *ws_X, double *op_all) {
  const int r = blockIdx.x;
  const int n = 4 * N, nr = n + 1;
  const int rows = 4 * N + 4;
  const double *Y = ws_X + (size_t)r * n * nr;
  double *op = op_all + (size_t)r * rows * nr;
  for (int idx = threadIdx.x; idx < rows * nr; idx += blockDim.x) {
    const int row = idx / nr, col = idx % nr;
    double v;
    if (row < 2 * N) {
      const int m = row >> 1, tl = row & 1;
      const int c = (m < N / 2) ? (tl == 0 ? 0 : 2) : (tl == 0 ? 1 : 3);
      v = Y[(size_t)(4 * m + c) * nr + col];
    } else if (row < 2 * N + 4) {
      const int c = row - 2 * N;
      double acc = 0.0;
      for (int m = 0; m < N; ++m) acc += w[m] * Y[(size_t)(4 * m + c) * nr + col];
      v = acc;
    } else {
      const int p = row - 2 * N - 4;
      const int m = p >> 1, side = p & 1;
      v = Y[(size_t)(4 * m + 2 + side) * nr + col];
    }
    op[idx] = v;
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
// two level-k rows).  Layout and use: oci_step.hip, "The structured apply".
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
  double *cf = coef + (size_t)idx * kCoef;
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
