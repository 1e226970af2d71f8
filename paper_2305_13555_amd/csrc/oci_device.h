// Device-side data structures and helpers shared by the OCI / SI kernels.
//
// Layouts (all FP64, row-major):
//   out  [J+2][2N]  outgoing angular flux of every cell, one buffer per
//                   iterate of a step (modulo the buffer count);
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
//   phi  [J][4]     scalar flux (k,L), (k,R), (k+1/2,L), (k+1/2,R), one buffer
//                   per iterate like out.
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

// Step control block, one per context, in device memory.  Every field has
// one writer (the first thread of work-group 0 of some launch, or the host
// between launches), and a launch only relies on values written by earlier
// launches: the kernel boundary orders them.  No kernel uses device-scope
// fences or atomics (on this GPU a device-scope release after a kernel's
// writes costs far more than a kernel boundary).
struct StepCtl {
  int32_t total0;        // iterations completed before this step (bookkeeping only)
  int32_t accepted;      // written by the iteration launch that decides the step
  int32_t status;        // kRunning from the step start; the decision once taken
  int32_t step_parity;   // psi buffer holding psi_{k-1/2}
  int32_t stalled;       // a queued step was not decided within its launches
  int32_t fin_accepted;  // the step's outcome, written by the end-of-step kernel
  int32_t fin_status;    //   (read by later launches and the host only, never by
                         //   the launch that writes it)
  int32_t open;          // the open step (its index in the solve) and the buffer its
  int32_t base_buf;      //   first iterate read: written by that iteration launch,
                         //   read by the end of the step
  int32_t cur;           // index of the next step to open (written by the host at
                         //   the start of a solve and by the end of a decided step)
  int32_t psi_base;      // psi buffer of step 0 of the current solve (host)
  int32_t fin_buf;       // iterate buffer holding the last decided step's accepted
                         //   iterate (written with fin_accepted)
  int32_t pad;
  double e_last;         // e of the accepted iterate (-1: undefined)
  double e_prev;         // source iteration: e of the previous iterate
  double fin_e;
  double fin_e_prev;     // e of the iterate before the accepted one (-1: undefined)
};

// Iterate buffers: two rings of nbuf, one per step parity (half h holds
// buffers h*nbuf .. h*nbuf+nbuf-1), then two for source iteration.  Iterate
// l >= 1 of a step of half h writes ring slot l % nbuf of that half and reads
// slot (l-1) % nbuf, except iterate 1, which reads the previous step's
// accepted iterate (buffer fin_buf, in the other half or a source-iteration
// buffer): a step never overwrites the iterate it started from, and no
// iteration launch but the first needs device data to pick its buffers.

// Per-step record of a queued solve.
struct StepRecord {
  int32_t accepted;
  int32_t status;
  double e_last;
  double e_prev;   // e of the iterate before the accepted one (-1: undefined)
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

// Wave reductions with DPP lane moves (vector ALU operands; a shuffle through
// ds_bpermute costs an LDS round trip per step).  Every lane of the wave must
// be active.  The steps: swap lanes within quads (xor 1, xor 2), mirror
// within half rows and rows (each lane then holds its 16-lane row's result),
// then row 3 combines with row 2 (row_bcast:15) and with rows 0-1
// (row_bcast:31), so lane 63 holds the wave's result, read back as a
// wave-uniform value.  The order is fixed: the same on every run.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ int dpp_i32(int v) {
  // (lanes of rows outside ROW_MASK get an unspecified value: only lane 63,
  // whose row every step includes, carries the result)
  return __builtin_amdgcn_mov_dpp(v, CTRL, ROW_MASK, 0xf, false);
}
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = dpp_i32<CTRL, ROW_MASK>((int)(b & 0xffffffffll));
  const int hi = dpp_i32<CTRL, ROW_MASK>((int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane63_f64(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
// Lane `src` of a wave-uniform index: its value, wave-uniform.
__device__ __forceinline__ double lane_f64(double v, int src) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

template <class Op>
__device__ __forceinline__ double wave_reduce(double v, Op op) {
  v = op(v, dpp_f64<0xB1>(v));          // quad_perm [1,0,3,2]
  v = op(v, dpp_f64<0x4E>(v));          // quad_perm [2,3,0,1]
  v = op(v, dpp_f64<0x141>(v));         // row_half_mirror
  v = op(v, dpp_f64<0x140>(v));         // row_mirror
  v = op(v, dpp_f64<0x142, 0xa>(v));    // row_bcast:15 (rows 1, 3)
  v = op(v, dpp_f64<0x143, 0xc>(v));    // row_bcast:31 (rows 2, 3)
  return lane63_f64(v);
}

__device__ __forceinline__ double wave_max(double v) {
  return wave_reduce(v, [](double x, double y) { return fmax(x, y); });
}

// Sum over the wave in a fixed order (the same on every run).
__device__ __forceinline__ double wave_sum(double v) {
  return wave_reduce(v, [](double x, double y) { return x + y; });
}

__device__ __forceinline__ int wave_or(int v) {
  v |= dpp_i32<0xB1>(v);
  v |= dpp_i32<0x4E>(v);
  v |= dpp_i32<0x141>(v);
  v |= dpp_i32<0x140>(v);
  v |= dpp_i32<0x142, 0xa>(v);
  v |= dpp_i32<0x143, 0xc>(v);
  return __builtin_amdgcn_readlane(v, 63);
}

// e_l = max|phi^(l) - phi^(l-1)| / max|phi^(l)| (0/0 -> 0, x/0 -> inf).
__device__ __forceinline__ double rel_change(double dphi, double phimax) {
  if (phimax == 0.0) return dphi == 0.0 ? 0.0 : __builtin_inf();
  return dphi / phimax;
}

// Stopping rule for iterate l (1-based) given its residual maxima and the e
// of iterate l-1 (-1 if undefined).  first_defined is the first iterate
// whose e exists (2 for OCI: its first iterate has no predecessor in the
// step; 1 for SI).  Returns the status and stores e_l (or -1) in *e_out.
__device__ inline int stop_rule(int l, double dphi, double phimax, int nonfinite,
                                double e_before, int first_defined, double tol, int strict,
                                int max_iters, double *e_out) {
  double e = -1.0;
  int done = kRunning;
  if (nonfinite || !(dphi == dphi) || !(phimax == phimax)) {
    done = kNonFinite;
  } else if (l >= first_defined) {
    e = rel_change(dphi, phimax);
    if (e <= tol) {
      if (!strict) {
        done = kConverged;
      } else if (e_before >= 0.0) {
        double rho = e_before == 0.0 ? 0.0 : e / e_before;
        rho = fmin(fmax(rho, 0.0), 0.9999);
        if (e * rho / (1.0 - rho) <= tol) done = kConverged;
      }
    }
  }
  if (done == kRunning && l >= max_iters) done = kIterLimit;
  *e_out = e;
  return done;
}

// The same rule from e_l itself (NaN when iterate l is not finite; the value
// is ignored for l < first_defined).
__device__ inline int stop_rule_e(int l, double e, double e_before, int first_defined, double tol,
                                  int strict, int max_iters) {
  if (e != e) return kNonFinite;
  int done = kRunning;
  if (l >= first_defined && e <= tol) {
    if (!strict) {
      done = kConverged;
    } else if (e_before >= 0.0) {
      double rho = e_before == 0.0 ? 0.0 : e / e_before;
      rho = fmin(fmax(rho, 0.0), 0.9999);
      if (e * rho / (1.0 - rho) <= tol) done = kConverged;
    }
  }
  if (done == kRunning && l >= max_iters) done = kIterLimit;
  return done;
}

// max that propagates NaN (a non-finite residual travels as NaN).
__device__ __forceinline__ double nan_max(double a, double b) {
  return (a != a || a > b) ? a : b;
}

__device__ __forceinline__ double wave_nan_max(double v) {
  return wave_reduce(v, [](double x, double y) { return nan_max(x, y); });
}

// Reduction over each 16-lane row of the wave in a fixed order; every lane
// of a row receives its row's result (four DPP steps, no cross-row moves).
template <class Op>
__device__ __forceinline__ double row_reduce16(double v, Op op) {
  v = op(v, dpp_f64<0xB1>(v));    // quad_perm [1,0,3,2]
  v = op(v, dpp_f64<0x4E>(v));    // quad_perm [2,3,0,1]
  v = op(v, dpp_f64<0x141>(v));   // row_half_mirror
  v = op(v, dpp_f64<0x140>(v));   // row_mirror
  return v;
}

__device__ __forceinline__ double row_sum16(double v) {
  return row_reduce16(v, [](double x, double y) { return x + y; });
}

// Residual records: one double2 per tile or block, (max|phi^(l) - phi^(l-1)|,
// max|phi^(l)|), the first set to NaN when any value of phi^(l) is not
// finite.  Slot s of a record array holds iterate l with l % 3 == s.
//
// Work-group reduction of n records: each thread's first kRecBatch records are
// loaded by rec_issue (so the loads can start at kernel entry) and combined
// with the rest by rec_finish into out[0..1] in LDS (ends with a barrier; every
// thread of the work-group must take part).
constexpr int kRecBatch = 4;
struct RecRegs {
  double2 v[kRecBatch];
};

__device__ __forceinline__ void rec_issue(RecRegs &r, const double2 *rec, int n) {
#pragma unroll
  for (int q = 0; q < kRecBatch; ++q) {
    const int i = threadIdx.x + q * blockDim.x;
    r.v[q] = i < n ? rec[i] : make_double2(0.0, 0.0);
  }
}

__device__ inline void rec_finish(const RecRegs &r, const double2 *rec, int n, double *out,
                                  double *scratch) {
  double d = 0.0, f = 0.0;
#pragma unroll
  for (int q = 0; q < kRecBatch; ++q) {
    d = nan_max(d, r.v[q].x);
    f = nan_max(f, r.v[q].y);
  }
  // the rest eight records per thread at a time (eight loads in flight)
  int i = threadIdx.x + kRecBatch * blockDim.x;
  for (; i + 7 * (int)blockDim.x < n; i += 8 * blockDim.x) {
    double2 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = rec[i + u * blockDim.x];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      d = nan_max(d, v[u].x);
      f = nan_max(f, v[u].y);
    }
  }
  for (; i < n; i += blockDim.x) {
    const double2 v = rec[i];
    d = nan_max(d, v.x);
    f = nan_max(f, v.y);
  }
  d = wave_nan_max(d);
  f = wave_nan_max(f);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, W = blockDim.x >> 6;
  if (lane == 0) {
    scratch[wave * 2 + 0] = d;
    scratch[wave * 2 + 1] = f;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < W; ++w) {
      d = nan_max(d, scratch[w * 2 + 0]);
      f = nan_max(f, scratch[w * 2 + 1]);
    }
    out[0] = d;
    out[1] = f;
  }
  __syncthreads();
}

}  // namespace ocik
