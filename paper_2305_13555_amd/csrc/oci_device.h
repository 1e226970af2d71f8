// Device-side data structures and helpers shared by the OCI / SI kernels.
//
// Layouts (all FP64, row-major):
//   out  [J+2][2N]  outgoing angular flux of every cell, ping-pong pair;
//                   row g = cell + 1, rows 0 and J+1 are ghost cells that
//                   hold the boundary values (vacuum: 0; incident: the given
//                   flux; reflecting: filled in LDS from the boundary cell).
//                   Entry 2m+t, t = 0 level k, 1 level k+1/2: for m < N/2
//                   (mu < 0) the left-half flux psi_{m,t,j,L}, which leaves
//                   through the left edge; for m >= N/2 the right-half flux
//                   psi_{m,t,j,R}, which leaves through the right edge
//                   (upstream closure).
//   inc_j (never stored): entries 0..N-1 from out_{j+1}, N..2N-1 from
//                   out_{j-1}: exactly the incident fluxes of c^- and c^+.
//   psi_prev / psi_next [J][2N]  time-edge state, entry 2m+s (s = L, R).
//   phi  [J][4]     scalar flux (k,L), (k,R), (k+1/2,L), (k+1/2,R), ping-pong.
//   gh   [J][Mt*16] per-step constant part of [out; phi] (see oci_step.hip).
//   operators: per region, packed in MFMA A-fragment order (see pack_frag).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ocik {

constexpr int kWave = 64;
constexpr int kTileCells = 16;    // cells per work-group tile (one MFMA column block)
constexpr int kMaxWaves = 8;      // waves per work-group in the GEMM kernels

typedef double d4 __attribute__((ext_vector_type(4)));

struct RegionDev {
  int32_t j0, nc;   // first cell, number of cells
  double dx, sig, sigs, q;
};

struct TileDev {
  int32_t region, c0, nc, pad;   // cells c0 .. c0+nc-1, all in one region, nc <= 16
};

// Iteration control word, one per context, in device memory.
struct StepState {
  int32_t it;        // iterations completed in the current step
  int32_t done;      // 0 running, 1 converged, 2 iteration limit, 3 non-finite
  uint32_t arrive;   // tiles that finished the current launch
  int32_t total;     // iterations since the last state reset (ping-pong parity)
  int32_t step_parity;  // which psi buffer holds psi_{k-1/2} in the current step
  int32_t pad;
  double e_last;     // e of the last iterate (-1: undefined)
  double e_prev;     // e of the iterate before it (-1: undefined)
};

enum { kRunning = 0, kConverged = 1, kIterLimit = 2, kNonFinite = 3 };
enum { kBcVacuum = 0, kBcReflect = 1, kBcIncident = 2 };

// D(16x16) += A(16x4) * B(4x16), FP64.  Lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; it receives D[l/16 + 4*i][l%16] in element i (for the f64
// variant the four accumulator elements of a lane are rows 4 apart).
// The kernels put cells on the rows (A = the tile's incident fluxes, one cell
// per row) and operator rows on the columns (B = the packed operator), so
// for a fixed element i the 16 lanes of a row group hold 16 consecutive
// output rows of one cell: loads and stores are contiguous per cell.
__device__ __forceinline__ d4 mfma16x16x4(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return v;
}

__device__ __forceinline__ int wave_or(int v) {
  for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ void store_agent(double *p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double load_agent(const double *p) {
  return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Shared stopping decision, taken by the last tile to finish an iteration.
// dphi = max|phi^(l) - phi^(l-1)|, phimax = max|phi^(l)|, nonfinite flag.
// first_defined: the first iteration (1-based) whose e is defined
// (2 for OCI, 1 for SI).
__device__ inline void decide(StepState *st, double dphi, double phimax, int nonfinite,
                              int max_iters, double tol, int strict, int first_defined) {
  const int l = st->it + 1;
  double e = -1.0;
  int done = kRunning;
  if (nonfinite || !(dphi == dphi) || !(phimax == phimax)) {
    done = kNonFinite;
  } else if (l >= first_defined) {
    if (phimax == 0.0) e = (dphi == 0.0) ? 0.0 : __builtin_inf();
    else e = dphi / phimax;
    if (e <= tol) {
      if (!strict) {
        done = kConverged;
      } else if (st->e_last >= 0.0) {
        const double prev = st->e_last;
        double rho = prev == 0.0 ? 0.0 : e / prev;
        rho = fmin(fmax(rho, 0.0), 0.9999);
        if (e * rho / (1.0 - rho) <= tol) done = kConverged;
      }
    }
  }
  if (done == kRunning && l >= max_iters) done = kIterLimit;
  st->e_prev = st->e_last;
  st->e_last = e;
  st->it = l;
  st->total = st->total + 1;
  st->arrive = 0;
  __threadfence();
  st->done = done;
}

}  // namespace ocik
