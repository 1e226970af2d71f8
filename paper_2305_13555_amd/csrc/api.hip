// Host driver behind the C ABI declared in include/oci.h.
//
// One context = one slab problem bound to one HIP stream.  oci_setup builds
// every region's operator on the GPU.  An OCI time step is the step-start
// kernel (per-step constant), L iteration launches (each decides the previous
// iterate from the residual records the launch before it left, and exits at
// once once the step is decided), and the end-of-step kernel, which decides
// the last iterate itself when no launch did.  Every argument of these
// kernels is static (the step index and buffers come from the device control
// block), so whole steps are replayed from cached HIP graphs.  oci_solve and
// oci_step queue windows of steps without waiting, L = the iteration count of
// the latest completed window; a step not decided within its L launches
// stalls the queue on the device and the host resumes it.  Source iteration
// runs one step at a time with host-read decisions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstddef>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "oci.h"
#include "oci_kernels.h"
#include "plan.h"
#include "corrector_internal.h"

using namespace ocik;

namespace {

thread_local std::string g_last_error;

using ocip::kMaxBatch;           // iteration launches per replayed batch
static_assert(kMaxBatch + 1 <= ocik::kMaxRing, "the end of step holds one ring of e values");
constexpr int kMaxInner = 64;   // FP32 inner iterations per correction (mixed precision)

}  // namespace

struct oci_ctx {
  hipStream_t stream = nullptr;
  int N = 0, J = 0, R = 0, bcl = 0, bcr = 0, max_iters = 0, strict = 0;
  double tol = 0.0, a = 0.0;
  std::vector<double> mu, w;
  std::vector<int> cells;
  std::vector<double> ghost_left, ghost_right;   // [2N] each
  int Mt = 0, Met = 0, Mto = 0, ntiles = 0, grid = 0, W_it = 1, W_ed = 1, W_pv = 1;
  size_t lds_it = 0, lds_pv = 0, lds_ed = 0;
  int si_blocks = 0, si_segs = 1;
  bool si_lane = false;   // the angle-lane sweep (N/2 a power of two, N <= 128)
  int si_nseg = 1;        // its segments
  double2 *d_segin = nullptr;
  Affine *d_chmap = nullptr;
  std::vector<void *> allocs;
  double *d_mu = nullptr, *d_w = nullptr;
  RegionDev *d_regions = nullptr;
  TileDev *d_tiles = nullptr;
  int *d_cell_region = nullptr;
  double *d_op = nullptr;
  double *d_fi = nullptr, *d_fp = nullptr, *d_cp = nullptr;
  size_t fi_stride = 0, fp_stride = 0, cp_stride = 0;
  double *d_gh = nullptr, *d_outb = nullptr, *d_phib = nullptr, *d_dec = nullptr;
  int nbuf = 3;                              // ring slots per half (buffers: 2*nbuf + 2)
  size_t out_stride = 0, phi_stride = 0;
  double *d_psi[2] = {nullptr, nullptr}, *d_phi_res = nullptr, *d_partial = nullptr;
  double *d_ainv = nullptr, *d_contrib = nullptr, *d_lag = nullptr, *d_si_partial = nullptr;
  double *d_coef = nullptr;
  double *d_phig = nullptr;   // [R][4][2N] scalar-flux rows of G, plain
  Affine *d_segmap = nullptr;
  StepCtl *d_ctl = nullptr;
  StepCtl *h_ctl = nullptr;                  // pinned host copy of the control block
  StepRecord *d_rec = nullptr, *h_rec = nullptr;
  int rec_cap = 0;
  int parity = 0;
  int64_t steps = 0;
  bool have_flux = false;
  int last_si_iters = 0;
  hipGraphExec_t si_graph[kMaxBatch + 1] = {};    // indexed by batch length
  hipEvent_t ev0 = nullptr, ev1 = nullptr, evA = nullptr, evB = nullptr;
  hipEvent_t evW[2][2] = {};                 // start / end of the windows in flight
  struct StepGraph {
    int L, G, half, begin, m, fuse;
    double *phi;
    hipGraphExec_t exec;
  };
  std::vector<StepGraph> step_graphs;        // G whole steps of L iteration launches
  bool gh_valid = false;                     // gh holds P psi_{k-1/2} + p for the next step
  int batch_hint = 0;                        // iteration launches per queued step
  int window = 1;                            // steps of the next queued window
  bool quad_override = false;
  int *d_bad = nullptr;                      // set by the operator build: singular system
  // mixed precision: FP64 iterates every other launch (rstep 2) with FP32
  // correction solves of m_inner iterations between them
  bool mixed = false;
  int rstep = 1, m_inner = 2;
  int pre_reduce = 0;   // the end of step reads the last iterate's e from k_reduce_rec
  // inner-count search: FP64 iterates per step seen at m_inner, the count
  // before a trial decrease and what it gave, no further decreases
  int m_q = 0, m_prev = 0, m_prev_q = 0;
  bool m_locked = false;
  bool m_fixed = false;   // set by oci_set_inner_iterations: no search
  float *d_fi32 = nullptr, *d_dlt = nullptr, *d_dphi32 = nullptr;
  size_t lds_in = 0, lds_in2 = 0;
  void *fn_inner2 = nullptr;   // two inner iterations per launch
  // kernels for the chosen operator batch width CH
  int CH = 16;
  void *fn_begin = nullptr, *fn_iter = nullptr, *fn_end = nullptr, *fn_inner = nullptr;
  void *fn_end_nf = nullptr;   // the end of step without the fused iterate
  void *fn_iter2 = nullptr;   // two iterates per launch (plain FP64 batches)
  size_t lds_it2 = 0;
  void *fn_iterK[5] = {};     // [3], [4]: three and four iterates per launch (N = 8 .. 64)
  size_t lds_itK[5] = {};
  int kimax = 2;              // most iterates per launch (the active cap)
  bool fuse_end = true;       // ends of queued steps compute the next step's iterate 1
  int kibuilt = 2;            // most iterates per launch this problem allows
  // learned corrections inside the iteration (oci_set_corrector)
  oci_corrector *corr = nullptr;
  int corr_first = 0, corr_period = 0, corr_in = 8;
  float *d_lx = nullptr, *d_ly = nullptr;       // corrector input [8][J], output [4][J]
  double *d_bak_out = nullptr, *d_bak_phi = nullptr;   // the corrected iterate, as it was
  double *h_dec = nullptr;                      // pinned host copy of dec
  std::string err;
  StepArgs sa{};
  SiArgs si{};
};

#define OCI_CK(ctx, call)                                                             \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) {                                                           \
      char b_[256];                                                                   \
      snprintf(b_, sizeof b_, "%s failed: %s", #call, hipGetErrorString(e_));         \
      (ctx)->err = b_;                                                                \
      g_last_error = b_;                                                              \
      return e_ == hipErrorOutOfMemory ? OCI_ENOMEM : OCI_EDEVICE;                    \
    }                                                                                 \
  } while (0)

static int fail(oci_ctx *c, int code, const std::string &msg) {
  if (c) c->err = msg;
  g_last_error = msg;
  return code;
}

template <class T>
static int dalloc(oci_ctx *c, T **p, size_t count) {
  void *q = nullptr;
  OCI_CK(c, hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)));
  c->allocs.push_back(q);
  *p = static_cast<T *>(q);
  return OCI_OK;
}

static int validate(const oci_problem *p, std::string *why) {
  auto bad = [&](const char *m) { *why = m; return OCI_EINVAL; };
  if (!p) return bad("problem is NULL");
  const int N = p->n_angles;
  if (N < 2 || N > OCI_MAX_ANGLES || (N & 1))
    return bad("n_angles must be even and in [2, 256] (odd Gauss-Legendre sets contain mu = 0)");
  if ((p->mu == nullptr) != (p->w == nullptr)) return bad("mu and w must be given together");
  if (p->mu) {
    for (int m = 0; m < N; ++m) {
      if (!(std::isfinite(p->mu[m]) && std::isfinite(p->w[m]) && p->w[m] > 0.0))
        return bad("quadrature weights must be positive and finite");
      if (p->mu[m] == 0.0 || std::fabs(p->mu[m]) > 1.0) return bad("mu must be nonzero, |mu| <= 1");
      if (m > 0 && !(p->mu[m] > p->mu[m - 1])) return bad("mu must be ascending");
      if (std::fabs(p->mu[m] + p->mu[N - 1 - m]) > 1e-12) return bad("mu must be mirror-symmetric");
    }
  }
  if (p->n_regions < 1 || !p->cells || !p->width || !p->sigma_t || !p->sigma_s || !p->source)
    return bad("n_regions >= 1 and the region arrays are required");
  long long J = 0;
  for (int r = 0; r < p->n_regions; ++r) {
    if (p->cells[r] < 1) return bad("every region needs >= 1 cell");
    if (!(p->width[r] > 0.0) || !std::isfinite(p->width[r])) return bad("region width must be > 0");
    if (!(p->sigma_t[r] > 0.0) || !std::isfinite(p->sigma_t[r])) return bad("sigma_t must be > 0");
    if (!(p->sigma_s[r] >= 0.0) || !std::isfinite(p->sigma_s[r])) return bad("sigma_s must be >= 0");
    if (!(p->source[r] >= 0.0) || !std::isfinite(p->source[r])) return bad("source must be >= 0");
    J += p->cells[r];
  }
  if (J > (1LL << 28)) return bad("too many cells");
  if (!(p->dt > 0.0) || !std::isfinite(p->dt)) return bad("dt must be > 0");
  if (!(p->speed > 0.0)) return bad("speed must be > 0 (inf for steady)");
  for (int s = 0; s < 2; ++s) {
    const int bc = s ? p->bc_right : p->bc_left;
    const double *inc = s ? p->inc_right : p->inc_left;
    if (bc < OCI_BC_VACUUM || bc > OCI_BC_INCIDENT) return bad("unknown boundary condition");
    if (bc == OCI_BC_INCIDENT) {
      if (!inc) return bad("incident boundary needs its [N/2] flux array");
      for (int i = 0; i < N / 2; ++i)
        if (!std::isfinite(inc[i])) return bad("incident flux must be finite");
    }
  }
  if (!(p->tol >= 0.0)) return bad("tol must be >= 0");
  if (p->max_iters < 1) return bad("max_iters must be >= 1");
  if (p->precision != OCI_PREC_FP64 && p->precision != OCI_PREC_FP32)
    return bad("precision must be OCI_PREC_FP64 or OCI_PREC_FP32");
  if (p->precision == OCI_PREC_FP32 && (p->flags & OCI_FLAG_STRICT))
    return bad("OCI_FLAG_STRICT needs OCI_PREC_FP64");
  if (p->flags & ~(OCI_FLAG_STRICT | OCI_FLAG_COMPACT)) return bad("unknown flags");
  if (p->psi0) {
    for (long long i = 0; i < J * N * 2; ++i)
      if (!std::isfinite(p->psi0[i])) return bad("psi0 must be finite");
  }
  return OCI_OK;
}

static int upload_ghosts(oci_ctx *c) {
  const int K = 2 * c->N;
  for (int b = 0; b < 2 * c->nbuf + 2; ++b) {
    double *o = c->d_outb + (size_t)b * c->out_stride;
    OCI_CK(c, hipMemcpyAsync(o, c->ghost_left.data(), K * sizeof(double), hipMemcpyHostToDevice,
                             c->stream));
    OCI_CK(c, hipMemcpyAsync(o + (size_t)(c->J + 1) * K, c->ghost_right.data(), K * sizeof(double),
                             hipMemcpyHostToDevice, c->stream));
  }
  return OCI_OK;
}

// Cold iterate: zero outgoing fluxes (cell rows; the boundary rows of every
// iterate buffer are set once at setup and never written) and scalar flux in
// buffer 0, zero lagged reflection, control block cleared (accepted iterate
// in buffer 0).
// (psi: also clear the time edge psi[0].)
static int reset_iterate(oci_ctx *c, bool psi = false) {
  static_assert(sizeof(StepCtl) % sizeof(double) == 0, "the control block clears as doubles");
  const int K = 2 * c->N;
  ZeroRanges z{};
  z.p[0] = c->d_outb + K;
  z.n[0] = (size_t)c->J * K;
  z.p[1] = c->d_phib;
  z.n[1] = (size_t)c->J * 4;
  z.p[2] = c->d_lag;
  z.n[2] = (size_t)2 * c->N;
  z.p[3] = reinterpret_cast<double *>(c->d_ctl);
  z.n[3] = sizeof(StepCtl) / sizeof(double);
  z.count = 4;
  if (psi) {
    z.p[4] = c->d_psi[0];
    z.n[4] = (size_t)c->J * K;
    z.count = 5;
  }
  hipLaunchKernelGGL(k_zero, dim3(256), dim3(256), 0, c->stream, z);
  OCI_CK(c, hipGetLastError());
  c->last_si_iters = 0;
  c->gh_valid = false;
  c->batch_hint = 0;
  c->window = 1;
  return OCI_OK;
}

// The first batch of a source-iteration step as a replayable graph: `count`
// iterations of sweep, reduce and decide launches.
static int build_si_graph(oci_ctx *c, int count) {
  hipGraphExec_t *slot = &c->si_graph[count];
  if (*slot) return OCI_OK;
  hipGraph_t g;
  OCI_CK(c, hipGraphCreate(&g, 0));
  hipGraphNode_t prev = nullptr;
  auto add = [&](void *fn, dim3 grid, dim3 block, size_t lds, void **args) -> hipError_t {
    hipKernelNodeParams kp{};
    kp.func = fn;
    kp.gridDim = grid;
    kp.blockDim = block;
    kp.sharedMemBytes = (unsigned)lds;
    kp.kernelParams = args;
    kp.extra = nullptr;
    hipGraphNode_t node;
    hipError_t e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
    if (e == hipSuccess) prev = node;
    return e;
  };
  hipError_t e = hipSuccess;
  for (int i = 1; i <= count && e == hipSuccess; ++i) {
    int node = i, cb = 0;
    void *args[] = {&c->si, &node, &cb};
    if (c->si_lane) {
      e = add((void *)k_si_smaps, dim3(c->si_nseg, 2), dim3(256), 0, args);
      if (e == hipSuccess) e = add((void *)k_si_enter, dim3(c->N / 2), dim3(256), 0, args);
      if (e == hipSuccess) e = add((void *)k_si_lsweep, dim3(c->si_nseg, 2), dim3(256), 0, args);
    } else {
      e = add((void *)k_si_maps, dim3(c->N / 2, c->si_segs), dim3(256), 0, args);
      if (e == hipSuccess) e = add((void *)k_si_sweep, dim3(c->N / 2, c->si_segs), dim3(256), 0, args);
    }
    if (e == hipSuccess) e = add((void *)k_si_reduce, dim3(c->si_blocks), dim3(256), 0, args);
    if (e == hipSuccess) e = add((void *)k_si_decide, dim3(1), dim3(256), 0, args);
  }
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(c, OCI_EDEVICE, std::string("hipGraphAddKernelNode: ") + hipGetErrorString(e));
  }
  e = hipGraphInstantiate(slot, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    *slot = nullptr;
    return fail(c, OCI_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  return OCI_OK;
}


// Build and pack every region's operator (region table, mu, w and a already
// on the device / in the context).
static int build_operators(oci_ctx *c) {
  const int N = c->N, R = c->R;
  int *d_bad = c->d_bad;
  OCI_CK(c, hipMemsetAsync(d_bad, 0, sizeof(int), c->stream));
  // every per-region table (A_m^{-1}, the cell operator and its packed
  // forms) in one launch; a region's work spread over nb work-groups
  SetupArgs q;
  q.regions = c->d_regions;
  q.mu = c->d_mu;
  q.w = c->d_w;
  q.N = N;
  q.Mt = c->Mt;
  q.a = c->a;
  q.ainv = c->d_ainv;
  q.coef = c->d_coef;
  q.phig = c->d_phig;
  q.op = c->d_op;
  q.frag_it = c->d_fi;
  q.frag_pv = c->d_fp;
  q.frag_it32 = c->mixed ? c->d_fi32 : nullptr;
  q.frag_stride = c->fi_stride;
  q.c_pv = c->d_cp;
  q.cvec_stride = c->cp_stride;
  q.bad = d_bad;
  const int nb = std::max(1, std::min(16, (256 + R - 1) / R));
  hipLaunchKernelGGL(k_region_setup, dim3(R, nb), dim3(256), (size_t)(32 * N + 4) * sizeof(double),
                     c->stream, q);
  OCI_CK(c, hipGetLastError());
  int bad = 0;
  OCI_CK(c, hipMemcpyAsync(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  OCI_CK(c, hipStreamSynchronize(c->stream));
  if (bad) return fail(c, OCI_EINVAL, "a region's cell matrix A - S is singular");
  return OCI_OK;
}

static void drop_step_graphs(oci_ctx *c) {
  // a queued window may still be running one of them
  if (!c->step_graphs.empty()) (void)hipStreamSynchronize(c->stream);
  for (auto &g : c->step_graphs) (void)hipGraphExecDestroy(g.exec);
  c->step_graphs.clear();
}

static void drop_graphs(oci_ctx *c) {
  drop_step_graphs(c);
  for (int i = 0; i <= kMaxBatch; ++i) {
    if (c->si_graph[i]) (void)hipGraphExecDestroy(c->si_graph[i]);
    c->si_graph[i] = nullptr;
  }
}

extern "C" int oci_setup(const oci_problem *p, void *hip_stream, oci_ctx **out) {
  if (!out) return fail(nullptr, OCI_EINVAL, "out is NULL");
  *out = nullptr;
  std::string why;
  if (validate(p, &why) != OCI_OK) return fail(nullptr, OCI_EINVAL, why);

  oci_ctx *c = new oci_ctx();
  c->stream = static_cast<hipStream_t>(hip_stream);
  const int N = p->n_angles, K = 2 * N, R = p->n_regions;
  c->N = N;
  c->R = R;
  c->bcl = p->bc_left;
  c->bcr = p->bc_right;
  c->tol = p->tol;
  c->max_iters = p->max_iters;
  c->strict = (p->flags & OCI_FLAG_STRICT) ? 1 : 0;
  c->mixed = p->precision == OCI_PREC_FP32;
  c->rstep = c->mixed ? 2 : 1;
  c->a = std::isinf(p->speed) ? 0.0 : 1.0 / (p->speed * p->dt);
  c->mu.resize(N);
  c->w.resize(N);
  c->quad_override = p->mu != nullptr;
  if (p->mu) {
    std::copy(p->mu, p->mu + N, c->mu.begin());
    std::copy(p->w, p->w + N, c->w.begin());
  } else {
    oci_gauss_legendre(N, c->mu.data(), c->w.data());
  }
  // region table and 16-cell tiles (a tile never straddles a region)
  std::vector<RegionDev> regions(R);
  std::vector<TileDev> tiles;
  std::vector<int> cell_region;
  int j0 = 0;
  for (int r = 0; r < R; ++r) {
    const int nc = p->cells[r];
    regions[r] = RegionDev{j0, nc, p->width[r] / nc, p->sigma_t[r], p->sigma_s[r], p->source[r]};
    for (int t0 = 0; t0 < nc; t0 += kTileCells)
      tiles.push_back(TileDev{r, j0 + t0, std::min(kTileCells, nc - t0), 0});
    cell_region.insert(cell_region.end(), nc, r);
    c->cells.push_back(nc);
    j0 += nc;
  }
  const int J = j0;
  c->J = J;
  c->ntiles = (int)tiles.size();
  c->grid = c->ntiles;   // one work-group per tile
  {
    // work-group order: the hardware dispatches work-groups round-robin over
    // the 8 XCDs, so the work-groups b = x, x+8, ... of XCD x take a
    // contiguous run of tiles (a region's operator in few L2s, neighbouring
    // tiles in the same L2)
    std::vector<TileDev> by_block(tiles.size());
    size_t next = 0;
    for (int x = 0; x < 8; ++x)
      for (int b = x; b < c->ntiles; b += 8) by_block[b] = tiles[next++];
    tiles.swap(by_block);
  }
  c->Mt = (2 * N + 4 + 15) / 16;
  c->Met = (2 * N + 15) / 16;
  c->Mto = (2 * N + 15) / 16;
  // at most four waves per work-group: the hardware places a work-group's
  // waves from the first SIMD of a CU onwards, so with five waves the first
  // SIMD fills first and fewer work-groups stay resident than registers
  // allow.  The iteration splits its scalar-flux dot products over W threads,
  // so there W is a power of two.
  c->W_it = std::min(c->Mto, 4);
  c->W_pv = std::min(c->Mt, 4);
  c->W_ed = std::min(c->Met, 4);
  const int P = K + 2;
  c->lds_it = (size_t)(kTileCells + 2) * P * sizeof(double);
  c->lds_it2 = (size_t)(kBlkA + kBlkB) * P * sizeof(double);
  c->lds_pv = (size_t)kTileCells * P * sizeof(double);
  c->lds_ed = (size_t)(2 * kTileCells + 2) * P * sizeof(double);
  c->si_blocks = (J * 4 + 255) / 256;
  // source-iteration sweep segments: about two cells per thread of a
  // 256-thread work-group, at most 64 segments
  c->si_segs = std::max(1, std::min(64, (J + 511) / 512));
  // the angle-lane sweep: 256 threads = N/2 angles x C chunks per segment,
  // about four cells per chunk, at most 512 segments
  c->si_lane = N <= 128 && ((N / 2) & (N / 2 - 1)) == 0;
  if (c->si_lane) {
    const int C = 256 / (N / 2);
    c->si_nseg = (int)std::max<long long>(1, std::min<long long>(512, ((long long)J + 4 * C - 1) / (4 * C)));
  }
  c->ghost_left.assign(K, 0.0);
  c->ghost_right.assign(K, 0.0);
  if (p->bc_left == OCI_BC_INCIDENT)
    for (int i = 0; i < N / 2; ++i) {
      const int m = N / 2 + i;
      c->ghost_left[2 * m] = c->ghost_left[2 * m + 1] = p->inc_left[i];
    }
  if (p->bc_right == OCI_BC_INCIDENT)
    for (int m = 0; m < N / 2; ++m) c->ghost_right[2 * m] = c->ghost_right[2 * m + 1] = p->inc_right[m];

  int rc = OCI_OK;
  auto cleanup = [&](int code) {
    oci_destroy(c);
    return code;
  };
#define OCI_TRY(x)                    \
  do {                                \
    rc = (x);                         \
    if (rc != OCI_OK) {               \
      g_last_error = c->err;          \
      return cleanup(rc);             \
    }                                 \
  } while (0)

  const int n = 4 * N, nr = n + 1, oprows = 4 * N + 4;
  c->fi_stride = (size_t)c->Mt * (K / 4) * 64;
  c->fp_stride = c->fi_stride;
  c->cp_stride = (size_t)c->Mt * 16;
  OCI_TRY(dalloc(c, &c->d_mu, N));
  OCI_TRY(dalloc(c, &c->d_w, N));
  OCI_TRY(dalloc(c, &c->d_regions, R));
  OCI_TRY(dalloc(c, &c->d_tiles, c->ntiles));
  OCI_TRY(dalloc(c, &c->d_cell_region, J));
  OCI_TRY(dalloc(c, &c->d_op, (size_t)R * oprows * nr));
  OCI_TRY(dalloc(c, &c->d_fi, (size_t)R * c->fi_stride));
  OCI_TRY(dalloc(c, &c->d_fp, (size_t)R * c->fp_stride));
  OCI_TRY(dalloc(c, &c->d_cp, (size_t)R * c->cp_stride));
  OCI_TRY(dalloc(c, &c->d_gh, (size_t)J * c->Mt * 16));
  // one buffer per iterate of a queued batch (at most kMaxBatch launches) in
  // each of two rings, one per step parity, within a memory budget
  c->out_stride = (size_t)(J + 2) * K;
  c->phi_stride = (size_t)J * 4;
  {
    const size_t per = (c->out_stride + c->phi_stride) * sizeof(double);
    // 1 GiB of rings per context (so that many contexts fit side by side),
    // but at least 9 slots: batches of up to 8 iterates per step
    // (OCI_FLAG_COMPACT: 64 MiB and at least 7 slots, for many contexts at once)
    const bool compact = (p->flags & OCI_FLAG_COMPACT) != 0;
    const size_t budget = compact ? (size_t)64 << 20 : (size_t)1 << 30;
    const size_t min_slots = compact ? 7 : 9;
    c->nbuf = (int)std::max<size_t>(min_slots,
                                    std::min<size_t>(kMaxBatch + 1, budget / (2 * per)));
  }
  const size_t nb_all = 2 * (size_t)c->nbuf + 2;   // two rings, two source-iteration buffers
  OCI_TRY(dalloc(c, &c->d_outb, nb_all * c->out_stride));
  OCI_TRY(dalloc(c, &c->d_phib, nb_all * c->phi_stride));
  OCI_TRY(dalloc(c, &c->d_dec, (size_t)c->nbuf));
  for (int b = 0; b < 2; ++b) OCI_TRY(dalloc(c, &c->d_psi[b], (size_t)J * K));
  OCI_TRY(dalloc(c, &c->d_phi_res, (size_t)J * 4));
  OCI_TRY(dalloc(c, &c->d_partial, (size_t)2 * c->nbuf * c->ntiles * 2));
  OCI_TRY(dalloc(c, &c->d_ainv, (size_t)R * N * 16));
  OCI_TRY(dalloc(c, &c->d_coef, (size_t)R * N * kCoef));
  OCI_TRY(dalloc(c, &c->d_phig, (size_t)R * 8 * N));
  OCI_TRY(dalloc(c, &c->d_contrib, (size_t)(c->si_lane ? 2 : N / 2) * J * 4));
  OCI_TRY(dalloc(c, &c->d_lag, (size_t)2 * N));
  OCI_TRY(dalloc(c, &c->d_segmap, (size_t)(N / 2) * std::max(c->si_segs, c->si_nseg) * 2));
  if (c->si_lane) {
    OCI_TRY(dalloc(c, &c->d_segin, (size_t)(N / 2) * c->si_nseg * 2));
    OCI_TRY(dalloc(c, &c->d_chmap, (size_t)256 * c->si_nseg * 2));
  }
  OCI_TRY(dalloc(c, &c->d_si_partial, (size_t)3 * c->si_blocks * 4));
  OCI_TRY(dalloc(c, &c->d_ctl, 1));
  if (c->mixed) {
    OCI_TRY(dalloc(c, &c->d_fi32, (size_t)R * c->fi_stride));
    OCI_TRY(dalloc(c, &c->d_dlt, (size_t)3 * c->out_stride));
    OCI_TRY(dalloc(c, &c->d_dphi32, (size_t)J * 4));
    // the correction's ghost rows stay zero (boundary values are constants)
    if (hipMemsetAsync(c->d_dlt, 0, (size_t)3 * c->out_stride * sizeof(float), c->stream) !=
        hipSuccess)
      return cleanup(fail(c, OCI_EDEVICE, "hipMemsetAsync failed"));
  }
  {
    void *h = nullptr;
    if (hipHostMalloc(&h, sizeof(StepCtl), hipHostMallocDefault) != hipSuccess)
      return cleanup(fail(c, OCI_ENOMEM, "hipHostMalloc failed"));
    c->h_ctl = static_cast<StepCtl *>(h);
  }
  if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
      hipEventCreate(&c->evA) != hipSuccess || hipEventCreate(&c->evB) != hipSuccess ||
      hipEventCreate(&c->evW[0][0]) != hipSuccess || hipEventCreate(&c->evW[0][1]) != hipSuccess ||
      hipEventCreate(&c->evW[1][0]) != hipSuccess || hipEventCreate(&c->evW[1][1]) != hipSuccess)
    return cleanup(fail(c, OCI_EDEVICE, "hipEventCreate failed"));

  auto up = [&](void *dst, const void *src, size_t bytes) -> int {
    OCI_CK(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream));
    return OCI_OK;
  };
  OCI_TRY(up(c->d_mu, c->mu.data(), N * sizeof(double)));
  OCI_TRY(up(c->d_w, c->w.data(), N * sizeof(double)));
  OCI_TRY(up(c->d_regions, regions.data(), R * sizeof(RegionDev)));
  OCI_TRY(up(c->d_tiles, tiles.data(), tiles.size() * sizeof(TileDev)));
  OCI_TRY(up(c->d_cell_region, cell_region.data(), (size_t)J * sizeof(int)));

  OCI_CK(c, hipFuncSetAttribute((const void *)k_region_setup,
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)((32 * N + 4) * sizeof(double))));
  OCI_TRY(dalloc(c, &c->d_bad, 1));
  OCI_TRY(build_operators(c));

  // ---- state ----
  OCI_TRY(upload_ghosts(c));
  OCI_TRY(reset_iterate(c));
  if (p->psi0) {
    OCI_TRY(up(c->d_psi[0], p->psi0, (size_t)J * K * sizeof(double)));
  } else {
    OCI_CK(c, hipMemsetAsync(c->d_psi[0], 0, (size_t)J * K * sizeof(double), c->stream));
  }
  OCI_CK(c, hipMemsetAsync(c->d_psi[1], 0, (size_t)J * K * sizeof(double), c->stream));
  OCI_CK(c, hipMemsetAsync(c->d_phi_res, 0, (size_t)J * 4 * sizeof(double), c->stream));

  // ---- kernel argument blocks ----
  StepArgs &s = c->sa;
  s.tiles = c->d_tiles;
  s.ntiles = c->ntiles;
  s.N = N;
  s.J = J;
  s.R = c->R;
  s.Mt = c->Mt;
  s.Met = c->Met;
  s.Mto = c->Mto;
  s.bcl = c->bcl;
  s.bcr = c->bcr;
  // mixed precision: the FP64 iterates are 1, 3, 5, ...; max_iters of them
  s.max_iters = c->mixed ? 2 * c->max_iters - 1 : c->max_iters;
  s.strict = c->strict;
  s.tol = c->tol;
  s.frag_it32 = c->d_fi32;
  s.dlt = c->d_dlt;
  s.dlt_stride = c->out_stride;
  s.dphi32 = c->d_dphi32;
  s.frag_it = c->d_fi;
  s.frag_it_stride = c->fi_stride;
  s.frag_pv = c->d_fp;
  s.frag_pv_stride = c->fp_stride;
  s.c_pv = c->d_cp;
  s.c_pv_stride = c->cp_stride;
  s.regions = c->d_regions;
  s.mu = c->d_mu;
  s.ainv = c->d_ainv;
  s.coef = c->d_coef;
  s.phig = c->d_phig;
  s.cell_region = c->d_cell_region;
  s.at = c->a;
  s.gh = c->d_gh;
  s.nbuf = c->nbuf;
  s.outb = c->d_outb;
  s.out_stride = c->out_stride;
  s.phib = c->d_phib;
  s.phi_stride = c->phi_stride;
  s.dec = c->d_dec;
  s.tiles_in_args = (c->ntiles <= kArgTiles && J < (1 << kArgTileCellBits) && R < 1024) ? 1 : 0;
  if (s.tiles_in_args)
    for (int i = 0; i < c->ntiles; ++i)
      s.tile_word[i] = pack_tile(tiles[i].region, tiles[i].c0, tiles[i].nc);
  s.psi0 = c->d_psi[0];
  s.psi1 = c->d_psi[1];
  s.phi_res = c->d_phi_res;
  s.partial = c->d_partial;
  s.ctl = c->d_ctl;
  s.rec = nullptr;
  SiArgs &q = c->si;
  q.N = N;
  q.J = J;
  q.bcl = c->bcl;
  q.bcr = c->bcr;
  q.max_iters = c->max_iters;
  q.strict = c->strict;
  q.tol = c->tol;
  q.a = c->a;
  q.regions = c->d_regions;
  q.cell_region = c->d_cell_region;
  q.mu = c->d_mu;
  q.w = c->d_w;
  q.ainv = c->d_ainv;
  q.own_buf = 2 * c->nbuf;
  q.out0 = c->d_outb + (size_t)q.own_buf * c->out_stride;
  q.out1 = q.out0 + c->out_stride;
  q.phi0 = c->d_phib + (size_t)q.own_buf * c->phi_stride;
  q.phi1 = q.phi0 + c->phi_stride;
  q.outb = c->d_outb;
  q.out_stride = c->out_stride;
  q.phib = c->d_phib;
  q.phi_stride = c->phi_stride;
  q.psi0 = c->d_psi[0];
  q.psi1 = c->d_psi[1];
  q.contrib = c->d_contrib;
  q.ncontrib = c->si_lane ? 2 : N / 2;
  q.lag = c->d_lag;
  q.segmap = c->d_segmap;
  q.segin = c->d_segin;
  q.chmap = c->d_chmap;
  q.nseg = c->si_nseg;
  q.phi_res = c->d_phi_res;
  q.partial = c->d_si_partial;
  q.nparts = c->si_blocks;
  q.ctl = c->d_ctl;

  // kernels for this N: operator fragments are fetched CH k-steps at a time
  c->CH = (N / 2 >= 16) ? 16 : (N / 2 >= 8 ? 8 : 4);
  // <CH, tiles in the kernel arguments, 16-byte operand reads (N % 8 == 0),
  // built for this N (common angle counts) or for any>
#define OCI_KERNEL(KN, CHV, ARGT)                                               \
  (N == 8 && CHV == 4      ? (void *)KN<4, ARGT, true, 8>                       \
   : N == 16 && CHV == 8   ? (void *)KN<8, ARGT, true, 16>                      \
   : N == 32 && CHV == 16  ? (void *)KN<16, ARGT, true, 32>                     \
   : N == 64 && CHV == 16  ? (void *)KN<16, ARGT, true, 64>                     \
   : N == 128 && CHV == 16 ? (void *)KN<16, ARGT, true, 128>                    \
   : N == 256 && CHV == 16 ? (void *)KN<16, ARGT, true, 256>                    \
   : N % 8 == 0            ? (void *)KN<CHV, ARGT, true, 0>                     \
                           : (void *)KN<CHV, ARGT, false, 0>)
#define OCI_PICK(CHV, ARGT)                                       \
  do {                                                            \
    c->fn_begin = OCI_KERNEL(k_step_begin, CHV, ARGT);            \
    c->fn_iter = OCI_KERNEL(k_oci_iterate, CHV, ARGT);            \
    c->fn_iter2 = OCI_KERNEL(k_oci_iterate2, CHV, ARGT);          \
    c->fn_end = OCI_KERNEL(k_step_end, CHV, ARGT);                \
    c->fn_end_nf = OCI_KERNEL(k_step_end_nf, CHV, ARGT);          \
  } while (0)
  if (s.tiles_in_args) {
    if (c->CH == 16) OCI_PICK(16, true);
    else if (c->CH == 8) OCI_PICK(8, true);
    else OCI_PICK(4, true);
  } else {
    if (c->CH == 16) OCI_PICK(16, false);
    else if (c->CH == 8) OCI_PICK(8, false);
    else OCI_PICK(4, false);
  }
#undef OCI_KERNEL
#undef OCI_PICK
  c->fn_inner = s.tiles_in_args ? (void *)k_oci_inner<true> : (void *)k_oci_inner<false>;
  c->fn_inner2 = s.tiles_in_args ? (void *)k_oci_inner2<true> : (void *)k_oci_inner2<false>;
  // three and four iterates per launch: built for N = 8, 16, 32 and 64 (from
  // N = 128 on the two LDS row blocks alone leave room for one work-group
  // per CU)
#define OCI_KERNELK(ARGT, KI)                                                   \
  (N == 8     ? (void *)k_oci_iterateK<4, ARGT, true, 8, KI>                    \
   : N == 16  ? (void *)k_oci_iterateK<8, ARGT, true, 16, KI>                   \
   : N == 32  ? (void *)k_oci_iterateK<16, ARGT, true, 32, KI>                  \
   : N == 64  ? (void *)k_oci_iterateK<16, ARGT, true, 64, KI>                  \
              : nullptr)
  // (the halo cells of a tile in its own region or the next one on their
  // side: no region narrower than ki-1 cells)
  const int min_cells = *std::min_element(c->cells.begin(), c->cells.end());
  for (int ki = 3; ki <= 4 && min_cells >= ki - 1; ++ki) {
    c->fn_iterK[ki] = s.tiles_in_args ? (ki == 3 ? OCI_KERNELK(true, 3) : OCI_KERNELK(true, 4))
                                      : (ki == 3 ? OCI_KERNELK(false, 3) : OCI_KERNELK(false, 4));
    // two row blocks, then the halo data: up to N = 32 the operator rows and
    // pair coefficients of three regions, from N = 64 on the tile's operator
    // rows only; and the halo cells' step constants
    const size_t halo_tables = N >= 64 ? (size_t)8 * N : (size_t)60 * N;
    c->lds_itK[ki] = ((size_t)2 * (kTileCells + 2 * ki) * (2 * N + 2) + halo_tables +
                      (size_t)2 * (ki - 1) * (2 * N + 4)) * sizeof(double);
    hipFuncAttributes fa{};
    // (at most 80 KiB of LDS, so that two work-groups share a CU's 160 KiB:
    // with one, the longer launches stop paying for themselves)
    if (c->fn_iterK[ki] && hipFuncGetAttributes(&fa, (const void *)c->fn_iterK[ki]) == hipSuccess &&
        c->lds_itK[ki] + fa.sharedSizeBytes <= (size_t)80 * 1024) {
      OCI_CK(c, hipFuncSetAttribute((const void *)c->fn_iterK[ki],
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)c->lds_itK[ki]));
      c->kimax = ki;
    }
  }
#undef OCI_KERNELK
  c->kibuilt = c->kimax;
  // from N = 128 on the two-iterate kernel (two row blocks of 2N+2 doubles,
  // 78 KiB of LDS at N = 128: two work-groups per CU) is slower per iterate
  // than single-iterate launches (four per CU): single iterates by default
  // (the tuner may still pick two)
  if (N >= 128) c->kimax = 1;
  // OCI_ITERATES_PER_LAUNCH (1 .. 4) caps the iterates of one launch
  if (const char *env = std::getenv("OCI_ITERATES_PER_LAUNCH")) {
    const int v = std::atoi(env);
    if (v >= 1 && v <= 4) c->kimax = std::min(c->kimax, v);
  }
  // past a few thousand tiles one reduction of the last iterate's records
  // beats every work-group of the end of step reducing them all
  c->pre_reduce = c->ntiles > 2048 ? 1 : 0;
  c->lds_in = (size_t)(kTileCells + 2) * (K + 4) * sizeof(float);
  // (two inner iterations per launch for N <= 128: rows, then the halo tables)
  c->lds_in2 = ((size_t)(2 * kTileCells + 6) * (K + 4) + 30 * N) * sizeof(float);
  if (N > 128) c->fn_inner2 = nullptr;
  // kernels with more than 64 KiB of dynamic LDS must say so
  OCI_CK(c, hipFuncSetAttribute((const void *)c->fn_iter,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds_it));
  OCI_CK(c, hipFuncSetAttribute((const void *)c->fn_iter2,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds_it2));
  OCI_CK(c, hipFuncSetAttribute((const void *)c->fn_begin,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds_pv));
  OCI_CK(c, hipFuncSetAttribute((const void *)c->fn_end,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds_ed));
  OCI_CK(c, hipFuncSetAttribute((const void *)c->fn_end_nf,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds_ed));
  if (c->fn_inner2)
    OCI_CK(c, hipFuncSetAttribute((const void *)c->fn_inner2,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds_in2));
  OCI_CK(c, hipStreamSynchronize(c->stream));
#undef OCI_TRY
  *out = c;
  return OCI_OK;
}

static int read_ctl(oci_ctx *c) {
  OCI_CK(c, hipMemcpyAsync(c->h_ctl, c->d_ctl, sizeof(StepCtl), hipMemcpyDeviceToHost, c->stream));
  OCI_CK(c, hipStreamSynchronize(c->stream));
  return OCI_OK;
}

// Resume a stalled queue: clear the stall flag so the open step can continue.
static int clear_stall(oci_ctx *c) {
  c->h_ctl->stalled = 0;
  OCI_CK(c, hipMemcpyAsync(&c->d_ctl->stalled, &c->h_ctl->stalled, sizeof(int32_t),
                           hipMemcpyHostToDevice, c->stream));
  return OCI_OK;
}

using ocip::resume_count;

// A later batch of a step: `count` launches after iterate cb (one by one:
// only needed when the first batch was too short).  For SI each iteration
// also decides.
static int launch_batch(oci_ctx *c, bool si, int cb, int count, int half = 0) {
  if (!ocip::batch_range_ok(cb, count))
    return fail(c, OCI_EDEVICE, "internal: iteration batch out of range");
  for (int i = 1; i <= count; ++i) {
    int node = i;
    if (!si) {
      int rstep = 1, nred = 1;
      void *args[] = {&c->sa, &node, &cb, &half, &rstep, &nred};
      OCI_CK(c, hipLaunchKernel(c->fn_iter, dim3(c->grid + 1), dim3(64 * c->W_it), args, c->lds_it,
                                c->stream));
    } else {
      void *args[] = {&c->si, &node, &cb};
      if (c->si_lane) {
        OCI_CK(c, hipLaunchKernel((const void *)k_si_smaps, dim3(c->si_nseg, 2), dim3(256), args, 0,
                                  c->stream));
        OCI_CK(c, hipLaunchKernel((const void *)k_si_enter, dim3(c->N / 2), dim3(256), args, 0,
                                  c->stream));
        OCI_CK(c, hipLaunchKernel((const void *)k_si_lsweep, dim3(c->si_nseg, 2), dim3(256), args,
                                  0, c->stream));
      } else {
        OCI_CK(c, hipLaunchKernel((const void *)k_si_maps, dim3(c->N / 2, c->si_segs), dim3(256),
                                  args, 0, c->stream));
        OCI_CK(c, hipLaunchKernel((const void *)k_si_sweep, dim3(c->N / 2, c->si_segs), dim3(256),
                                  args, 0, c->stream));
      }
      OCI_CK(c, hipLaunchKernel((const void *)k_si_reduce, dim3(c->si_blocks), dim3(256), args, 0,
                                c->stream));
      OCI_CK(c, hipLaunchKernel((const void *)k_si_decide, dim3(1), dim3(256), args, 0,
                                c->stream));
    }
  }
  return OCI_OK;
}

// A-posteriori error bound of an accepted iterate with e = e_l and
// e_prev = e_{l-1}: e rho / (1 - rho), rho = e / e_prev clamped to
// [0, 0.9999] (the strict stopping rule's bound); -1 when either is undefined.
static double error_bound(double e, double e_prev) {
  if (!(e >= 0.0) || !(e_prev >= 0.0)) return -1.0;
  double rho = e_prev == 0.0 ? 0.0 : e / e_prev;
  rho = std::min(std::max(rho, 0.0), 0.9999);
  return e * rho / (1.0 - rho);
}

static void fill_info(oci_step_info *info, int iterations, int status, double residual, double ms,
                      double iter_ms, int launches, double err_bound = -1.0,
                      int corrections = 0) {
  if (!info) return;
  info->iterations = iterations;
  info->status = status;
  info->residual = residual;
  info->ms = ms;
  info->iter_ms = iter_ms;
  info->launches = launches;
  info->corrections = corrections;
  info->err_bound = err_bound;
}

// A non-finite step is abandoned: psi_{k-1/2} is kept, the iterate restarts cold.
static int abandon_step(oci_ctx *c, oci_step_info *info, int iterations) {
  int rc = reset_iterate(c);
  OCI_CK(c, hipStreamSynchronize(c->stream));
  fill_info(info, iterations, OCI_ENONFINITE, -1.0, 0.0, 0.0, 0);
  if (rc) return rc;
  return fail(c, OCI_ENONFINITE, "the scalar flux became NaN or Inf");
}

// ---------------------------------------------------------------------------
// Source iteration: one step at a time, host-driven batches.
// ---------------------------------------------------------------------------
static int si_run(oci_ctx *c, oci_step_info *info) {
  c->gh_valid = false;   // psi_{k-1/2} changes under the OCI step start's gh
  OCI_CK(c, hipEventRecord(c->ev0, c->stream));
  const int nb = (int)std::min<size_t>(1024, ((size_t)c->J * 2 * c->N + 255) / 256);
  hipLaunchKernelGGL(k_si_begin, dim3(nb), dim3(256), 0, c->stream, c->si, c->parity);
  OCI_CK(c, hipGetLastError());
  int launched = 0, extra = 0, launches = 0;
  double iter_ms = 0.0;
  for (;;) {
    int count, rc;
    OCI_CK(c, hipEventRecord(c->evA, c->stream));
    if (launched == 0) {
      count = std::min(std::max(c->last_si_iters, 1), std::min(kMaxBatch, c->max_iters));
      rc = build_si_graph(c, count);
      if (rc) return rc;
      OCI_CK(c, hipGraphLaunch(c->si_graph[count], c->stream));
    } else {
      ++extra;
      count = resume_count(extra);
      rc = launch_batch(c, true, launched, count);
      if (rc) return rc;
    }
    OCI_CK(c, hipEventRecord(c->evB, c->stream));
    launched += count;
    rc = read_ctl(c);
    if (rc) return rc;
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, c->evA, c->evB);
    iter_ms += ms;
    launches += count;
    if (c->h_ctl->status != kRunning) break;
    if (launched > c->max_iters + 1)
      return fail(c, OCI_EDEVICE, "the step control block did not reach a decision");
  }
  const StepCtl st = *c->h_ctl;
  if (st.status == kNonFinite) return abandon_step(c, info, st.accepted);
  const int n = c->J * 4;
  hipLaunchKernelGGL(k_si_end, dim3(std::min(1024, (n + 255) / 256)), dim3(256), 0, c->stream,
                     c->si);
  OCI_CK(c, hipGetLastError());
  OCI_CK(c, hipEventRecord(c->ev1, c->stream));
  OCI_CK(c, hipEventSynchronize(c->ev1));
  float ms = 0.0f;
  (void)hipEventElapsedTime(&ms, c->ev0, c->ev1);
  c->last_si_iters = st.accepted;
  c->parity ^= 1;
  c->steps += 1;
  c->have_flux = true;
  const int status = st.status == kConverged ? OCI_OK : OCI_NOT_CONVERGED;
  fill_info(info, st.accepted, status, st.e_last, ms, iter_ms, launches,
            error_bound(st.e_last, st.e_prev));
  return status;
}

// ---------------------------------------------------------------------------
// One-cell inversion: queued steps.
// ---------------------------------------------------------------------------
constexpr int kWindow = 32;  // steps per queued window (one graph of whole steps)
constexpr int kColdBatch = 8;  // launches of a step with no previous step to go by
constexpr int kColdOuter = 3;  // mixed precision: FP64 iterates of such a step

// Per-step records of a solve; the step graphs hold the device pointer, so
// growing the buffer drops them.
// The records live in pinned, device-mapped host memory: the end of step
// writes them there, and the host reads a window's records once its end
// event has completed (no copy on the stream between windows).
static int grow_records(oci_ctx *c, int n) {
  if (n <= c->rec_cap) return OCI_OK;
  drop_step_graphs(c);
  if (c->h_rec) (void)hipHostFree(c->h_rec);
  if (c->h_dec) (void)hipHostFree(c->h_dec);
  c->d_rec = nullptr;
  c->h_rec = nullptr;
  c->rec_cap = 0;
  c->sa.rec = nullptr;
  const int cap = std::max(n, 1024);
  OCI_CK(c, hipHostMalloc((void **)&c->h_rec, cap * sizeof(StepRecord), hipHostMallocMapped));
  OCI_CK(c, hipHostGetDevicePointer((void **)&c->d_rec, c->h_rec, 0));
  c->rec_cap = cap;
  c->sa.rec = c->d_rec;
  return OCI_OK;
}

// G whole steps as one replayable graph: with `begin`, a step start (gh of
// the first step; each end of step computes the next step's gh), then per
// step L iteration launches and the end of step (which writes phi_out[step]
// when phi is given).  Every argument is static: the step index and psi
// buffer come from the control block, the ring half alternates from `half`.
//
// Mixed precision: L is the number of FP64 iterates per step (1, 3, .., 2L-1);
// before each FP64 iterate after the first, m_inner FP32 inner iterations,
// the last of which forms the even iterate the FP64 one starts from.
static int step_graph(oci_ctx *c, int L, int G, int half, int begin, double *phi,
                      hipGraphExec_t *out) {
  const int m = c->mixed ? c->m_inner : 0;
  const int fz = c->fuse_end ? 1 : 0;
  for (auto &g : c->step_graphs)
    if (g.L == L && g.G == G && g.half == half && g.begin == begin && g.m == m &&
        g.fuse == fz && g.phi == phi) {
      *out = g.exec;
      return OCI_OK;
    }
  if (c->step_graphs.size() >= 32) drop_step_graphs(c);
  hipGraph_t g;
  OCI_CK(c, hipGraphCreate(&g, 0));
  hipGraphNode_t prev = nullptr;
  // (extra: work-groups past the tiles; the iteration kernels have one that
  // reduces the previous launch's residual records)
  auto add = [&](void *fn, int W, size_t lds, void **args, int extra = 0) -> hipError_t {
    hipKernelNodeParams kp{};
    kp.func = fn;
    kp.gridDim = dim3(c->grid + extra);
    kp.blockDim = dim3(64 * W);
    kp.sharedMemBytes = (unsigned)lds;
    kp.kernelParams = args;
    kp.extra = nullptr;
    hipGraphNode_t node;
    hipError_t e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
    if (e == hipSuccess) prev = node;
    return e;
  };
  hipError_t e = hipSuccess;
  void *bargs[] = {&c->sa};
  if (begin) e = add(c->fn_begin, c->W_pv, c->lds_pv, bargs);
  int rstep = c->rstep;
  // the end of every step but the graph's last also computes iterate 1 of
  // the next step (needs L >= 2, so that the next step still has a launch of
  // its own to open it; mixed precision: FP64 iterate 1 with its defect, and
  // the next step's first inner iteration opens it)
  const bool fuse_ok = L >= 2 && fz;
  int last_n = 1;   // iterates of the step's last launch
  for (int s = 0; s < G && e == hipSuccess; ++s) {
    int h = (half + s) & 1;
    if (c->mixed) {
      const int ostart = (s > 0 && fuse_ok) ? 2 : 1;
      for (int o = ostart; o <= L && e == hipSuccess; ++o) {
        // the m inner iterations: two per launch, a single one first when m is odd
        for (int i = 1, n = 1; o > 1 && i <= m && e == hipSuccess; ++n) {
          const int lv = c->fn_inner2 && (m - i + 1) % 2 == 0 ? 2 : 1;
          int nn = n, ly = i + lv - 1 == m ? 2 * (o - 1) : 0;
          int opens = (o == ostart && i == 1) ? 1 : 0;
          void *iargs[] = {&c->sa, &nn, &ly, &h, &opens};
          e = lv == 2 ? add(c->fn_inner2, c->W_it, c->lds_in2, iargs)
                      : add(c->fn_inner, c->W_it, c->lds_in, iargs);
          i += lv;
        }
        // (iterate 1's outgoing fluxes feed nothing when a correction follows;
        // the last FP64 iterate's defect only a resumed step, which forms it)
        int node = 2 * o - 1, cb = 0, nred = 1;
        int rmode = rstep | (o == 1 && L >= 2 ? 4 : 0) | (o == L ? 8 : 0);
        void *args[] = {&c->sa, &node, &cb, &h, &rmode, &nred};
        if (e == hipSuccess) e = add(c->fn_iter, c->W_it, c->lds_it, args, 1);
      }
    } else {
      // iterates start .. L in launches of up to kimax iterates each; after a
      // fused end of step (every step of the graph but the first) iterate 1
      // is already done
      const int start = (s > 0 && fuse_ok) ? 2 : 1;
      int prev_n = 1;
      for (int o = start; o <= L && e == hipSuccess;) {
        const int k = std::min(L - o + 1, c->kimax);
        int node = o, cb = 0, nred = prev_n;
        if (k == 1) {
          void *args[] = {&c->sa, &node, &cb, &h, &rstep, &nred};
          e = add(c->fn_iter, c->W_it, c->lds_it, args, 1);
        } else if (k == 2) {
          void *args[] = {&c->sa, &node, &cb, &h, &nred};
          e = add(c->fn_iter2, c->W_it, c->lds_it2, args, 1);
        } else {
          void *args[] = {&c->sa, &node, &cb, &h, &nred};
          e = add(c->fn_iterK[k], c->W_it, c->lds_itK[k], args, 1);
        }
        prev_n = k;
        o += k;
      }
      last_n = prev_n;
    }
    const bool fuse = fuse_ok && s + 1 < G;
    int first = 1, last = c->mixed ? 2 * L - 1 : L, nred = c->mixed ? 1 : last_n;
    int pre = c->pre_reduce, mode = pre | (nred << 1) | (fuse ? 16 : 0) | (fuse && c->mixed ? 32 : 0);
    if (e == hipSuccess && pre) {
      void *rargs[] = {&c->sa, &last, &nred, &h};
      hipKernelNodeParams kp{};
      kp.func = (void *)k_reduce_rec;
      kp.gridDim = dim3(nred);   // (one work-group per trailing iterate)
      kp.blockDim = dim3(256);
      kp.sharedMemBytes = 0;
      kp.kernelParams = rargs;
      kp.extra = nullptr;
      hipGraphNode_t node;
      e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
      if (e == hipSuccess) prev = node;
    }
    if (e == hipSuccess) {
      void *eargs[] = {&c->sa, &phi, &first, &last, &h, &rstep, &mode};
      e = add(fuse ? c->fn_end : c->fn_end_nf, c->W_ed, c->lds_ed, eargs);
    }
  }
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(c, OCI_EDEVICE, std::string("hipGraphAddKernelNode: ") + hipGetErrorString(e));
  }
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess)
    return fail(c, OCI_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  c->step_graphs.push_back({L, G, half, begin, m, fz, phi, exec});
  *out = exec;
  return OCI_OK;
}

// Iterates queued for a step whose count is expected to be `want`: at most
// max_iters, within the iterate buffers.
// (Mixed precision: FP64 iterates, 2*batch-1 iterate buffers.)
static int step_batch(oci_ctx *c, int want) {
  const int cap = c->mixed ? c->nbuf / 2 : c->nbuf - 1;
  return std::max(1, std::min({want, c->max_iters, cap}));
}

// Iterations reported for an accepted iterate index (mixed: FP64 iterates) and
// the iteration launches of a queued step.
static int step_iterations(const oci_ctx *c, int accepted) {
  return c->mixed ? (accepted + 1) / 2 : accepted;
}
static int step_launches(const oci_ctx *c, int batch) {
  return c->mixed ? batch + (batch - 1) * c->m_inner : batch;
}

// Mixed precision: inner iterations per correction, from the most FP64
// iterates a completed window's steps took (q) with m_used inner iterations.  Four or more (three suffice
// at tol ~ 1e-10 when each correction gains the ~1e-6 that FP32 allows):
// double them.  Otherwise try one fewer; if that costs FP64 iterates, go back
// and stop decreasing.
static void tune_inner(oci_ctx *c, int q, int m_used) {
  if (c->m_fixed) return;
  if (m_used != c->m_inner) return;   // a window queued before the last change
  if (q >= 4) {
    if (c->m_inner < kMaxInner) c->m_inner = std::min(kMaxInner, 2 * c->m_inner);
    c->m_q = 0;
    c->m_prev = 0;
    c->m_locked = false;
    return;
  }
  if (c->m_prev && q > c->m_prev_q) {
    c->m_inner = c->m_prev;
    c->m_q = c->m_prev_q;
    c->m_prev = 0;
    c->m_locked = true;
    return;
  }
  c->m_q = q;
  c->m_prev = 0;
  if (!c->m_locked && c->m_inner > 1) {
    c->m_prev = c->m_inner;
    c->m_prev_q = q;
    c->m_inner -= 1;
  }
}

// Mixed precision: one more correction after FP64 iterate lprev (inner
// iterations, the last forming iterate lprev+1) and FP64 iterate lprev+2.
static int launch_outer(oci_ctx *c, int lprev, int half) {
  const int m = c->m_inner;
  for (int i = 1, n = 1; i <= m; ++n) {   // (as in step_graph)
    const int lv = c->fn_inner2 && (m - i + 1) % 2 == 0 ? 2 : 1;
    int nn = n, ly = i + lv - 1 == m ? lprev + 1 : 0, opens = 0;
    void *iargs[] = {&c->sa, &nn, &ly, &half, &opens};
    OCI_CK(c, hipLaunchKernel(lv == 2 ? c->fn_inner2 : c->fn_inner, dim3(c->grid),
                              dim3(64 * c->W_it), iargs, lv == 2 ? c->lds_in2 : c->lds_in,
                              c->stream));
    i += lv;
  }
  int node = lprev + 2, cb = 0, rstep = 2, nred = 1;
  void *args[] = {&c->sa, &node, &cb, &half, &rstep, &nred};
  OCI_CK(c, hipLaunchKernel(c->fn_iter, dim3(c->grid + 1), dim3(64 * c->W_it), args, c->lds_it,
                            c->stream));
  return OCI_OK;
}

static int launch_end(oci_ctx *c, double *phi_dev, int first, int last, int half) {
  // the end reads the records of iterates first .. last, one ring of them
  if (!ocip::end_range_ok(first, last, c->nbuf))
    return fail(c, OCI_EDEVICE, "internal: end of step over an iterate range out of bounds");
  // (single-iterate launches only: resumed steps)
  int rstep = c->rstep, pre = c->pre_reduce, nred = 1, mode = pre | 2;
  if (pre) {
    void *rargs[] = {&c->sa, &last, &nred, &half};
    OCI_CK(c, hipLaunchKernel((const void *)k_reduce_rec, dim3(nred), dim3(256), rargs, 0,
                              c->stream));
  }
  void *args[] = {&c->sa, &phi_dev, &first, &last, &half, &rstep, &mode};
  OCI_CK(c, hipLaunchKernel(c->fn_end_nf, dim3(c->grid), dim3(64 * c->W_ed), args, c->lds_ed,
                            c->stream));
  return OCI_OK;
}

// Queue steps first .. first+count-1 (whole-step graphs of `batch` iteration
// launches; step `first` uses ring half `half`) between two events; their
// records reach the host through mapped memory.
static int enqueue_window(oci_ctx *c, int first, int count, int batch, int half,
                          double *phi_dev, hipEvent_t ev_start, hipEvent_t ev_end) {
  OCI_CK(c, hipEventRecord(ev_start, c->stream));
  int left = count;
  while (left > 0) {
    int G = kWindow;   // whole steps per graph: 32, 16, 8, 4, 2 or 1
    while (G > left) G >>= 1;
    hipGraphExec_t exec;
    int rc = step_graph(c, batch, G, half, c->gh_valid ? 0 : 1, phi_dev, &exec);
    if (rc) return rc;
    c->gh_valid = true;
    OCI_CK(c, hipGraphLaunch(exec, c->stream));
    left -= G;
    half ^= G & 1;
  }
  OCI_CK(c, hipEventRecord(ev_end, c->stream));
  return OCI_OK;
}

static void complete_step(oci_ctx *c, int accepted) {
  c->parity ^= 1;
  c->steps += 1;
  c->have_flux = true;
}

// Resume step k (ring half = its psi parity) after its queued launches left it undecided: further
// iteration launches (1, 1, 2, 4, ... at a time) each followed by the end of
// step, until the end decides.  `launched` = iteration launches so far.
static int resume_step(oci_ctx *c, int launched, double *phi_dev, int *total_launches,
                       float *ms) {
  OCI_CK(c, hipEventRecord(c->ev0, c->stream));
  int extra = 0, launches = c->mixed ? step_launches(c, (launched + 1) / 2) : launched;
  for (;;) {
    int rc = clear_stall(c);
    if (rc) return rc;
    ++extra;
    if (c->mixed) {
      if (extra == 1) {   // the defect of the last queued FP64 iterate (not stored by it)
        int l = launched, h = c->parity;
        void *dargs[] = {&c->sa, &l, &h};
        OCI_CK(c, hipLaunchKernel((const void *)k_defect, dim3(1024), dim3(256), dargs, 0,
                                  c->stream));
      }
      rc = launch_outer(c, launched, c->parity);
      if (rc) return rc;
      launched += 2;
      launches += c->m_inner + 1;
      rc = launch_end(c, phi_dev, launched, launched, c->parity);
    } else {
      const int count = ocip::resumed_batch(extra, launched, c->max_iters, c->nbuf);
      rc = launch_batch(c, false, launched, count, c->parity);
      if (rc) return rc;
      launched += count;
      launches += count;
      rc = launch_end(c, phi_dev, launched - count + 1, launched, c->parity);
    }
    if (rc) return rc;
    rc = read_ctl(c);
    if (rc) return rc;
    if (!c->h_ctl->stalled || c->h_ctl->fin_status == kNonFinite) break;
    if (launched > c->sa.max_iters + 1)
      return fail(c, OCI_EDEVICE, "the step control block did not reach a decision");
  }
  OCI_CK(c, hipEventRecord(c->ev1, c->stream));
  OCI_CK(c, hipEventSynchronize(c->ev1));
  (void)hipEventElapsedTime(ms, c->ev0, c->ev1);
  *total_launches = launches;
  return OCI_OK;
}

// Steps 0 .. n_steps-1 of a solve are queued in windows of kWindow steps, two
// windows in flight, each step with the iteration count of the latest
// completed window as its launch count.  A step not decided within its
// launches stalls the queue on the device (the rest of the queue becomes
// no-ops); the host drains the stream, resumes that step and queues again
// from the next.  A step with no previous step to go by is queued alone.
// phi_dev may be null.
static int solve_queued(oci_ctx *c, int n_steps, double *phi_dev, oci_step_info *infos) {
  int rc = grow_records(c, n_steps);
  if (rc) return rc;
  // open the solve: step counter 0, psi buffer of step 0
  c->h_ctl->cur = 0;
  c->h_ctl->psi_base = c->parity;
  static_assert(offsetof(StepCtl, psi_base) == offsetof(StepCtl, cur) + sizeof(int32_t),
                "cur and psi_base are copied together");
  OCI_CK(c, hipMemcpyAsync(&c->d_ctl->cur, &c->h_ctl->cur, 2 * sizeof(int32_t),
                           hipMemcpyHostToDevice, c->stream));
  struct Win {
    int first, count, batch, ev, m;   // m: inner iterations (mixed precision)
  };
  Win wins[2];
  int nwin = 0, next_ev = 0;
  int worst = OCI_OK;
  int k = 0, q = 0;   // first step not complete, next step to queue
  while (k < n_steps) {
    // a cold step (no previous count) goes alone; nothing is queued behind it
    while (q < n_steps && nwin < 2 && c->batch_hint > 0) {
      const int batch = step_batch(c, c->batch_hint);
      // windows grow 1, 4, 16, .. kWindow steps, so that a count learnt from
      // few steps is not applied to many
      const int count = std::min(c->window, n_steps - q);
      c->window = std::min(kWindow, 4 * c->window);
      const int ev = next_ev;
      next_ev ^= 1;
      rc = enqueue_window(c, q, count, batch, c->parity ^ ((q - k) & 1), phi_dev,
                          c->evW[ev][0], c->evW[ev][1]);
      if (rc) return rc;
      wins[nwin++] = Win{q, count, batch, ev, c->m_inner};
      q += count;
    }
    if (nwin == 0) {
      const int batch = step_batch(c, c->mixed ? kColdOuter : kColdBatch);
      const int ev = next_ev;
      next_ev ^= 1;
      rc = enqueue_window(c, q, 1, batch, c->parity ^ ((q - k) & 1), phi_dev, c->evW[ev][0],
                          c->evW[ev][1]);
      if (rc) return rc;
      wins[nwin++] = Win{q, 1, batch, ev, c->m_inner};
      q += 1;
    }
    const Win w = wins[0];
    OCI_CK(c, hipEventSynchronize(c->evW[w.ev][1]));
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, c->evW[w.ev][0], c->evW[w.ev][1]);
    int done = w.first, hint = 0;
    while (done < w.first + w.count && (c->h_rec[done].status == kConverged ||
                                        c->h_rec[done].status == kIterLimit))
      ++done;
    const int ndone = done - w.first;
    for (int s = w.first; s < done; ++s) {
      const StepRecord &r = c->h_rec[s];
      const int status = r.status == kConverged ? OCI_OK : OCI_NOT_CONVERGED;
      if (status == OCI_NOT_CONVERGED) worst = OCI_NOT_CONVERGED;
      // the window's stream time split evenly over its steps
      const double share = ms / w.count;
      fill_info(infos ? &infos[s] : nullptr, step_iterations(c, r.accepted), status, r.e_last,
                share, share, step_launches(c, w.batch),
                c->mixed ? -1.0 : error_bound(r.e_last, r.e_prev));
      complete_step(c, r.accepted);
      hint = std::max(hint, step_iterations(c, r.accepted));
    }
    k = done;
    if (ndone > 0) c->batch_hint = std::max(hint, 1);
    if (c->mixed && ndone > 0) tune_inner(c, hint, w.m);
    if (ndone == w.count) {
      wins[0] = wins[1];
      --nwin;
      continue;
    }
    // step k stalled: undecided after w.batch launches, or non-finite.  The
    // queue behind it is all no-ops; drain it and resume.
    OCI_CK(c, hipStreamSynchronize(c->stream));
    nwin = 0;
    rc = read_ctl(c);
    if (rc) return rc;
    if (c->h_ctl->fin_status == kNonFinite)
      return abandon_step(c, infos ? &infos[k] : nullptr, c->h_ctl->fin_accepted);
    int launches = 0;
    float rms = 0.0f;
    rc = resume_step(c, c->mixed ? 2 * w.batch - 1 : w.batch, phi_dev, &launches, &rms);
    if (rc) return rc;
    if (c->h_ctl->fin_status == kNonFinite)
      return abandon_step(c, infos ? &infos[k] : nullptr, c->h_ctl->fin_accepted);
    const StepCtl st = *c->h_ctl;
    const int status = st.fin_status == kConverged ? OCI_OK : OCI_NOT_CONVERGED;
    if (status == OCI_NOT_CONVERGED) worst = OCI_NOT_CONVERGED;
    fill_info(infos ? &infos[k] : nullptr, step_iterations(c, st.fin_accepted), status, st.fin_e,
              ms / w.count + rms, rms, launches,
              c->mixed ? -1.0 : error_bound(st.fin_e, st.fin_e_prev));
    complete_step(c, st.fin_accepted);
    c->batch_hint = std::max(step_iterations(c, st.fin_accepted), 1);
    if (c->mixed) tune_inner(c, c->batch_hint, c->m_inner);
    c->window = 1;
    ++k;
    q = k;
  }
  return worst;
}

// ---------------------------------------------------------------------------
// Host-driven steps: learned corrections inside the iteration, iterate history
// ---------------------------------------------------------------------------
// One OCI step in batches of single-iterate launches, each batch judged by an
// end of step (as a resumed step is).  With a corrector attached, iterate l =
// first, first + period, ... (plain, and not accepted) is corrected: the
// corrector predicts dphi from the scalar fluxes of iterates l-2 .. l, the
// iterate's scalar flux moves by dphi and its outgoing fluxes by the
// isotropic angular flux of that change (k_learn_apply), and iterate l+1 is
// the plain OCI iterate of that point.  It is kept when its change e_{l+1}
// is below rho e_l (rho = e_l / e_{l-1}: below what a plain iterate would
// reach, so the correction lowered the residual); otherwise iterate l is
// restored bit for bit, iterate l+1 recomputed from it, and the period to the
// next correction doubled (up to 1024 iterates; back to `period` after a kept
// one).  So a rejected correction leaves the plain sequence unchanged and an
// unhelpful corrector costs few attempts.  Every accepted iterate is a plain
// OCI iterate of its predecessor, judged by the stopping rule.  With hist
// (n_hist > 0) the scalar flux of iterates hist_first .. hist_first +
// n_hist - 1 (those computed) is copied out as they are formed.
static int host_step(oci_ctx *c, double *phi_dev, oci_step_info *info, double *hist, int n_hist,
                     bool hist_on_device, int hist_first = 1) {
  const int J = c->J, K = 2 * c->N, h = c->parity;
  c->h_ctl->cur = 0;
  c->h_ctl->psi_base = h;
  OCI_CK(c, hipMemcpyAsync(&c->d_ctl->cur, &c->h_ctl->cur, 2 * sizeof(int32_t),
                           hipMemcpyHostToDevice, c->stream));
  OCI_CK(c, hipEventRecord(c->ev0, c->stream));
  if (!c->gh_valid) {
    void *bargs[] = {&c->sa};
    OCI_CK(c, hipLaunchKernel(c->fn_begin, dim3(c->grid), dim3(64 * c->W_pv), bargs, c->lds_pv,
                              c->stream));
    c->gh_valid = true;
  }
  const size_t phin = (size_t)J * 4;
  const int hist_last = hist_first + n_hist - 1;
  auto copy_hist = [&](int l) -> int {
    if (!hist || l < hist_first || l > hist_last) return OCI_OK;
    OCI_CK(c, hipMemcpyAsync(hist + (size_t)(l - hist_first) * phin,
                             c->d_phib + (size_t)(h * c->nbuf + l % c->nbuf) * c->phi_stride,
                             phin * sizeof(double),
                             hist_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                             c->stream));
    return OCI_OK;
  };
  auto out_slot = [&](int l) { return c->d_outb + (size_t)(h * c->nbuf + l % c->nbuf) * c->out_stride; };
  auto phi_slot = [&](int l) { return c->d_phib + (size_t)(h * c->nbuf + l % c->nbuf) * c->phi_stride; };
  // plain iterates l0+1 .. l0+count, then the end of step over them
  auto plain = [&](int l0, int count) -> int {
    int rc = clear_stall(c);
    for (int i = 1; rc == OCI_OK && i <= count; ++i) {
      rc = launch_batch(c, false, l0 + i - 1, 1, h);
      if (rc == OCI_OK) rc = copy_hist(l0 + i);
    }
    if (rc == OCI_OK) rc = launch_end(c, phi_dev, l0 + 1, l0 + count, h);
    if (rc == OCI_OK) rc = read_ctl(c);
    return rc;
  };
  auto decided = [&]() { return !c->h_ctl->stalled || c->h_ctl->fin_status == kNonFinite; };
  int launched = 0, launches = 0, corrections = 0, rc = OCI_OK;
  int next_corr = c->corr ? c->corr_first : 0;
  int period = c->corr_period;   // doubled after each rejected correction (up to 1024)
  for (;;) {
    int count = (c->corr && next_corr > launched) ? next_corr - launched : kMaxBatch;
    if (hist && launched < hist_last) count = std::min(count, hist_last - launched);
    count = std::min({count, c->nbuf - 1, kMaxBatch, std::max(c->max_iters - launched, 1)});
    rc = plain(launched, count);
    if (rc) return rc;
    launched += count;
    launches += count;
    if (decided()) break;
    if (launched > c->max_iters + 1)
      return fail(c, OCI_EDEVICE, "the step control block did not reach a decision");
    if (!(c->corr && launched == next_corr && launched >= 3)) continue;
    const int l = launched;
    // the corrected point in slot l (its plain values kept for a restore)
    OCI_CK(c, hipMemcpyAsync(c->d_bak_out, out_slot(l) + K, (size_t)J * K * sizeof(double),
                             hipMemcpyDeviceToDevice, c->stream));
    OCI_CK(c, hipMemcpyAsync(c->d_bak_phi, phi_slot(l), phin * sizeof(double),
                             hipMemcpyDeviceToDevice, c->stream));
    double amp = 0.0;   // rho / (1 - rho) from the e of iterates l-1 and l
    if (c->corr_in == 12) {
      OCI_CK(c, hipMemcpyAsync(c->h_dec, c->d_dec, (size_t)c->nbuf * sizeof(double),
                               hipMemcpyDeviceToHost, c->stream));
      OCI_CK(c, hipStreamSynchronize(c->stream));
      const double e0 = c->h_dec[l % c->nbuf], em = c->h_dec[(l - 1) % c->nbuf];
      const double rho = em > 0.0 ? std::min(std::max(e0 / em, 0.0), 0.9999) : 0.0;
      amp = rho / (1.0 - rho);
    }
    const int nb = (int)std::min<size_t>(2048, (phin + 255) / 256);
    hipLaunchKernelGGL(k_learn_features, dim3(nb), dim3(256), 0, c->stream, c->sa, l, h,
                       c->corr_in, amp, c->d_lx);
    OCI_CK(c, hipGetLastError());
    rc = occ_infer32(c->corr, c->stream, c->d_lx, J, c->d_ly);
    if (rc) return fail(c, OCI_EDEVICE, "corrector inference failed");
    const int na = (int)std::min<size_t>(4096, ((size_t)J * c->N + 255) / 256);
    hipLaunchKernelGGL(k_learn_apply, dim3(na), dim3(256), 0, c->stream, c->sa, l, h, c->d_ly);
    OCI_CK(c, hipGetLastError());
    rc = plain(l, 1);
    if (rc) return rc;
    launches += 1;
    if (decided()) {   // iterate l+1 of the corrected point was accepted
      launched = l + 1;
      ++corrections;
      break;
    }
    OCI_CK(c, hipMemcpyAsync(c->h_dec, c->d_dec, (size_t)c->nbuf * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream));
    OCI_CK(c, hipStreamSynchronize(c->stream));
    const double e1 = c->h_dec[(l + 1) % c->nbuf], e0 = c->h_dec[l % c->nbuf];
    const double em = c->h_dec[(l - 1) % c->nbuf];
    const double rho = em > 0.0 ? std::min(std::max(e0 / em, 0.0), 1.0) : 1.0;
    if (e1 < rho * e0) {
      ++corrections;
      launched = l + 1;
      period = c->corr_period;
      next_corr = launched + period - 1;
      continue;
    }
    period = std::min(2 * period, 1024);
    next_corr = l + 1 + period - 1;
    // rejected: iterate l as it was, and its plain successor
    OCI_CK(c, hipMemcpyAsync(out_slot(l) + K, c->d_bak_out, (size_t)J * K * sizeof(double),
                             hipMemcpyDeviceToDevice, c->stream));
    OCI_CK(c, hipMemcpyAsync(phi_slot(l), c->d_bak_phi, phin * sizeof(double),
                             hipMemcpyDeviceToDevice, c->stream));
    rc = plain(l, 1);
    if (rc) return rc;
    launches += 1;
    launched = l + 1;
    if (decided()) break;
  }
  OCI_CK(c, hipEventRecord(c->ev1, c->stream));
  OCI_CK(c, hipEventSynchronize(c->ev1));
  float ms = 0.0f;
  (void)hipEventElapsedTime(&ms, c->ev0, c->ev1);
  const StepCtl st = *c->h_ctl;
  if (st.fin_status == kNonFinite) return abandon_step(c, info, st.fin_accepted);
  const int status = st.fin_status == kConverged ? OCI_OK : OCI_NOT_CONVERGED;
  fill_info(info, st.fin_accepted, status, st.fin_e, ms, ms, launches,
            error_bound(st.fin_e, st.fin_e_prev), corrections);
  complete_step(c, st.fin_accepted);
  c->batch_hint = std::max(st.fin_accepted, 1);
  c->window = 1;
  return status;
}

extern "C" int oci_set_corrector(oci_ctx *c, oci_corrector *k, int32_t first, int32_t period) {
  if (!c) return fail(nullptr, OCI_EINVAL, "context is NULL");
  if (!k) {
    c->corr = nullptr;
    return OCI_OK;
  }
  if (c->mixed) return fail(c, OCI_EINVAL, "learned corrections need OCI_PREC_FP64");
  if (first < 3 || period < 1)
    return fail(c, OCI_EINVAL, "corrections need first >= 3 and period >= 1");
  int ci = 0, co = 0;
  int64_t maxc = 0;
  if (occ_channels(k, &ci, &co, &maxc) != OCI_OK || (ci != 8 && ci != 12) || co != 4)
    return fail(c, OCI_EINVAL, "the corrector must map 8 or 12 input channels to 4");
  if (maxc < c->J) return fail(c, OCI_EINVAL, "the corrector takes fewer cells than the mesh has");
  if (!c->d_lx) {   // buffers of the first attached corrector, kept until oci_destroy
    OCI_CK(c, hipStreamSynchronize(c->stream));
    int rc = dalloc(c, &c->d_lx, (size_t)12 * c->J);
    if (rc == OCI_OK) rc = dalloc(c, &c->d_ly, (size_t)4 * c->J);
    if (rc == OCI_OK) rc = dalloc(c, &c->d_bak_out, (size_t)c->J * 2 * c->N);
    if (rc == OCI_OK) rc = dalloc(c, &c->d_bak_phi, (size_t)c->J * 4);
    if (rc) return rc;
    void *hp = nullptr;
    if (hipHostMalloc(&hp, kMaxRing * sizeof(double), hipHostMallocDefault) != hipSuccess)
      return fail(c, OCI_ENOMEM, "hipHostMalloc failed");
    c->h_dec = static_cast<double *>(hp);
  }
  c->corr = k;
  c->corr_first = first;
  c->corr_period = period;
  c->corr_in = ci;
  return OCI_OK;
}

extern "C" int oci_step_history(oci_ctx *c, int32_t first, int32_t n_hist, double *phi_hist,
                                int32_t on_device, oci_step_info *info) {
  if (!c) return fail(nullptr, OCI_EINVAL, "context is NULL");
  if (first < 1 || n_hist < 0 || (n_hist > 0 && !phi_hist))
    return fail(c, OCI_EINVAL, "bad history window or buffer");
  if (c->mixed) return fail(c, OCI_EINVAL, "iterate histories need OCI_PREC_FP64");
  oci_corrector *k = c->corr;
  c->corr = nullptr;   // plain iterates only
  const int rc = host_step(c, nullptr, info, phi_hist, n_hist, on_device != 0, first);
  c->corr = k;
  return rc;
}

extern "C" int oci_refactor(oci_ctx *c, const oci_problem *p) {
  if (!c) return fail(nullptr, OCI_EINVAL, "context is NULL");
  std::string why;
  if (validate(p, &why) != OCI_OK) return fail(c, OCI_EINVAL, why);
  if (p->n_angles != c->N || p->n_regions != c->R || p->bc_left != c->bcl ||
      p->bc_right != c->bcr || (p->mu != nullptr) != c->quad_override ||
      (p->precision == OCI_PREC_FP32) != c->mixed)
    return fail(c, OCI_EINVAL,
                "refactor needs the same angles, regions, boundary kinds and precision");
  for (int r = 0; r < c->R; ++r)
    if (p->cells[r] != c->cells[r]) return fail(c, OCI_EINVAL, "refactor needs the same cells");
  if (p->mu)
    for (int m = 0; m < c->N; ++m)
      if (p->mu[m] != c->mu[m] || p->w[m] != c->w[m])
        return fail(c, OCI_EINVAL, "refactor needs the same quadrature");
  std::vector<RegionDev> regions(c->R);
  int j0 = 0;
  for (int r = 0; r < c->R; ++r) {
    const int nc = c->cells[r];
    regions[r] = RegionDev{j0, nc, p->width[r] / nc, p->sigma_t[r], p->sigma_s[r], p->source[r]};
    j0 += nc;
  }
  OCI_CK(c, hipMemcpyAsync(c->d_regions, regions.data(), c->R * sizeof(RegionDev),
                           hipMemcpyHostToDevice, c->stream));
  c->a = std::isinf(p->speed) ? 0.0 : 1.0 / (p->speed * p->dt);
  c->tol = p->tol;
  c->max_iters = p->max_iters;
  c->strict = (p->flags & OCI_FLAG_STRICT) ? 1 : 0;
  const StepArgs sa0 = c->sa;
  const SiArgs si0 = c->si;
  c->sa.tol = c->si.tol = c->tol;
  c->si.max_iters = c->max_iters;
  c->sa.max_iters = c->mixed ? 2 * c->max_iters - 1 : c->max_iters;
  c->sa.strict = c->si.strict = c->strict;
  c->si.a = c->a;
  c->sa.at = c->a;
  // graphs hold copies of the argument blocks: rebuild them only if those changed
  if (std::memcmp(&sa0, &c->sa, sizeof sa0) != 0 || std::memcmp(&si0, &c->si, sizeof si0) != 0)
    drop_graphs(c);
  c->gh_valid = false;   // P and p change with the cross sections and dt
  return build_operators(c);
}

extern "C" int oci_step(oci_ctx *c, oci_step_info *info) {
  if (!c) return fail(nullptr, OCI_EINVAL, "context is NULL");
  if (c->corr) return host_step(c, nullptr, info, nullptr, 0, false);
  return solve_queued(c, 1, nullptr, info);
}

extern "C" int si_step(oci_ctx *c, oci_step_info *info) {
  if (!c) return fail(nullptr, OCI_EINVAL, "context is NULL");
  return si_run(c, info);
}

extern "C" int oci_solve(oci_ctx *c, int32_t n_steps, double *phi_out, int32_t phi_out_on_device,
                         oci_step_info *infos) {
  if (!c) return fail(nullptr, OCI_EINVAL, "context is NULL");
  if (n_steps < 0) return fail(c, OCI_EINVAL, "n_steps must be >= 0");
  if (n_steps == 0) return OCI_OK;
  if (c->corr && (phi_out == nullptr || phi_out_on_device)) {   // step by step, host-driven
    int worst = OCI_OK;
    for (int k = 0; k < n_steps; ++k) {
      const int rc = host_step(c, phi_out ? phi_out + (size_t)k * c->J * 4 : nullptr,
                               infos ? &infos[k] : nullptr, nullptr, 0, false);
      if (rc < 0) return rc;
      if (rc == OCI_NOT_CONVERGED) worst = OCI_NOT_CONVERGED;
    }
    return worst;
  }
  if (phi_out == nullptr || phi_out_on_device) return solve_queued(c, n_steps, phi_out, infos);
  // host output: step by step, copying each step's flux
  int worst = OCI_OK;
  const size_t per = (size_t)c->J * 4;
  for (int k = 0; k < n_steps; ++k) {
    int rc = oci_step(c, infos ? &infos[k] : nullptr);
    if (rc < 0) return rc;
    if (rc == OCI_NOT_CONVERGED) worst = OCI_NOT_CONVERGED;
    OCI_CK(c, hipMemcpyAsync(phi_out + k * per, c->d_phi_res, per * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream));
  }
  OCI_CK(c, hipStreamSynchronize(c->stream));
  return worst;
}

extern "C" int oci_solve_batch(oci_ctx **ctx, int32_t n_ctx, int32_t n_steps, double **phi_out,
                               int32_t phi_out_on_device, oci_step_info **infos,
                               int32_t n_threads) {
  if (!ctx || n_ctx < 1) return fail(nullptr, OCI_EINVAL, "need at least one context");
  if (n_steps < 0) return fail(nullptr, OCI_EINVAL, "n_steps must be >= 0");
  for (int i = 0; i < n_ctx; ++i) {
    if (!ctx[i]) return fail(nullptr, OCI_EINVAL, "context is NULL");
    for (int j = 0; j < i; ++j)
      if (ctx[j] == ctx[i]) return fail(nullptr, OCI_EINVAL, "contexts must be distinct");
  }
  const int T = std::max(1, std::min(n_ctx, n_threads > 0 ? n_threads : 16));
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(nullptr, OCI_EDEVICE, "hipGetDevice failed");
  std::vector<int> rc(n_ctx, OCI_OK);
  std::atomic<int> next(0);
  // each worker takes the next unsolved context: T problems progress at once
  auto work = [&]() {
    if (hipSetDevice(dev) != hipSuccess) return;
    for (;;) {
      const int i = next.fetch_add(1);
      if (i >= n_ctx) break;
      rc[i] = oci_solve(ctx[i], n_steps, phi_out ? phi_out[i] : nullptr, phi_out_on_device,
                        infos ? infos[i] : nullptr);
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < T; ++t) pool.emplace_back(work);
  work();
  for (auto &th : pool) th.join();
  if (next.load() < n_ctx) return fail(nullptr, OCI_EDEVICE, "hipSetDevice failed in a worker");
  int worst = OCI_OK;
  for (int i = 0; i < n_ctx; ++i) {
    if (rc[i] < 0) return rc[i];   // the context's own last error has the message
    if (rc[i] == OCI_NOT_CONVERGED) worst = OCI_NOT_CONVERGED;
  }
  return worst;
}

// ---------------------------------------------------------------------------
// Ensembles: one launch per iteration over the tiles of every problem
// ---------------------------------------------------------------------------
namespace {
struct EnsembleBufs {
  std::vector<void *> ptrs;
  void *host = nullptr;   // pinned staging of the per-batch tables
  ~EnsembleBufs() {
    for (void *q : ptrs) (void)hipFree(q);
    if (host) (void)hipHostFree(host);
  }
  template <class T>
  hipError_t alloc(T **p, size_t n) {
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T));
    if (e == hipSuccess) {
      ptrs.push_back(q);
      *p = static_cast<T *>(q);
    }
    return e;
  }
};
}  // namespace

extern "C" int oci_solve_ensemble(oci_ctx **ctx, int32_t n_ctx, int32_t n_steps,
                                  double **phi_out, oci_step_info **infos) {
  if (!ctx || n_ctx < 1) return fail(nullptr, OCI_EINVAL, "need at least one context");
  if (n_steps < 0) return fail(nullptr, OCI_EINVAL, "n_steps must be >= 0");
  for (int i = 0; i < n_ctx; ++i) {
    oci_ctx *c = ctx[i];
    if (!c) return fail(nullptr, OCI_EINVAL, "context is NULL");
    for (int j = 0; j < i; ++j)
      if (ctx[j] == c) return fail(nullptr, OCI_EINVAL, "contexts must be distinct");
    if (c->mixed || c->corr) return fail(c, OCI_EINVAL, "ensembles take plain FP64 contexts");
    if (c->N % 8) return fail(c, OCI_EINVAL, "ensembles take angle counts that are multiples of 8");
    if (c->parity != ctx[0]->parity)
      return fail(c, OCI_EINVAL, "ensemble contexts must be at the same step parity");
  }
  if (n_steps == 0) return OCI_OK;
  oci_ctx *c0 = ctx[0];
  const hipStream_t st = c0->stream;
  for (int i = 0; i < n_ctx; ++i) OCI_CK(c0, hipStreamSynchronize(ctx[i]->stream));
  // per problem: step records for the solve, step counter 0, psi buffer
  int cap = kMaxBatch;
  for (int i = 0; i < n_ctx; ++i) {
    oci_ctx *c = ctx[i];
    int rc = grow_records(c, n_steps);
    if (rc) return rc;
    c->h_ctl->cur = 0;   // (the device copies: kb_set_ctl below)
    c->h_ctl->psi_base = c->parity;
    cap = std::min(cap, c->nbuf - 1);
  }
  // the problems by angle count and iterates per launch: one class per pair
  // present, with the kernels built for that N (and its work-group sizes)
  // where there are, else the kernels for any N with 256 threads.  A problem
  // whose own launches may take three or four iterates (N = 8 .. 64, its
  // iterates-per-launch cap) runs that many per ensemble launch, else one.
  struct Cls {
    int N = 0, KI = 1, L = 0;
    void *fb = nullptr, *fi = nullptr, *fe = nullptr;
    dim3 bb, bi, be;
    size_t lb = 0, li = 0, le = 0;
    int nt_all = 0, nt_tiles = 0;
    int2 *d_qall = nullptr, *d_qtiles = nullptr;   // the current batch's queues
    size_t na = 0, nt = 0;                          // and their lengths
    int2 *d_all_full = nullptr, *d_tiles_full = nullptr;   // every problem's, uploaded once
    std::vector<int2> qall, qtiles;
  };
  std::vector<Cls> cls;
  std::vector<int> cls_of(n_ctx), kin(n_ctx, 1);
  for (int i = 0; i < n_ctx; ++i) {
    oci_ctx *c = ctx[i];
    const bool spec = c->N == 8 || c->N == 16 || c->N == 32 || c->N == 64 || c->N == 128;
    const int ki = (spec && c->N <= 64 && c->kimax >= 3) ? std::min(c->kimax, 4) : 1;
    kin[i] = ki;
    int k = 0;
    while (k < (int)cls.size() && !(cls[k].N == c->N && cls[k].KI == ki)) ++k;
    if (k == (int)cls.size()) {
      Cls q;
      q.N = c->N;
      q.KI = ki;
#define OCI_KB_PICK(CHV, NFV)                                  \
  do {                                                         \
    q.fb = (void *)kb_step_begin<CHV, NFV>;                    \
    q.fi = (void *)kb_oci_iterate<CHV, NFV>;                   \
    q.fe = (void *)kb_step_end<CHV, NFV>;                      \
  } while (0)
#define OCI_KB_PICKK(CHV, NFV)                                 \
  do {                                                         \
    OCI_KB_PICK(CHV, NFV);                                     \
    if (ki == 3) q.fi = (void *)kb_oci_iterateK<CHV, NFV, 3>;  \
    if (ki == 4) q.fi = (void *)kb_oci_iterateK<CHV, NFV, 4>;  \
  } while (0)
      switch (spec ? c->N : 0) {
        case 8: OCI_KB_PICKK(4, 8); break;
        case 16: OCI_KB_PICKK(8, 16); break;
        case 32: OCI_KB_PICKK(16, 32); break;
        case 64: OCI_KB_PICKK(16, 64); break;
        case 128: OCI_KB_PICK(16, 128); break;
        default: OCI_KB_PICK(4, 0); break;
      }
#undef OCI_KB_PICKK
#undef OCI_KB_PICK
      q.bb = dim3(spec ? 64 * c->W_pv : 256);
      q.bi = dim3(spec ? 64 * c->W_it : 256);
      q.be = dim3(spec ? 64 * c->W_ed : 256);
      q.lb = c->lds_pv;
      q.li = ki > 1 ? c->lds_itK[ki] : c->lds_it;
      q.le = c->lds_ed;
      cls.push_back(q);
    }
    cls_of[i] = k;
    cls[k].nt_all += ctx[i]->ntiles + 1;
    cls[k].nt_tiles += ctx[i]->ntiles;
  }
  // device tables: argument blocks, result pointers, the work queues
  EnsembleBufs db;
  StepArgs *d_probs = nullptr;
  double **d_phis = nullptr;
  int *d_plist = nullptr, *d_first = nullptr, *d_last = nullptr, *d_ki = nullptr;
  OCI_CK(c0, db.alloc(&d_ki, n_ctx));
  OCI_CK(c0, db.alloc(&d_probs, n_ctx));
  OCI_CK(c0, db.alloc(&d_phis, n_ctx));
  // a batch's tables (problem list, first, last, every class's queues) go to
  // the device in one transfer from one pinned staging buffer, each table at
  // an even offset (int2 queues); the host rewrites it only after the stream
  // has drained the batch before
  size_t pack_cap = 3 * ((size_t)n_ctx + 1);
  for (const Cls &q : cls) pack_cap += 2 * ((size_t)q.nt_all + q.nt_tiles);
  int *d_pack = nullptr;
  OCI_CK(c0, db.alloc(&d_pack, pack_cap));
  OCI_CK(c0, hipHostMalloc(&db.host, pack_cap * sizeof(int), hipHostMallocDefault));
  int *const h_pack = static_cast<int *>(db.host);
  // the queues of every problem (the batches planned at each step's start):
  // built and uploaded once
  {
    for (int i = 0; i < n_ctx; ++i) {
      Cls &q = cls[cls_of[i]];
      for (int t = 0; t <= ctx[i]->ntiles; ++t) q.qall.push_back(make_int2(i, t));
      for (int t = 0; t < ctx[i]->ntiles; ++t) q.qtiles.push_back(make_int2(i, t));
    }
    std::vector<int2> full;
    for (const Cls &q : cls) {
      full.insert(full.end(), q.qall.begin(), q.qall.end());
      full.insert(full.end(), q.qtiles.begin(), q.qtiles.end());
    }
    int2 *d_full = nullptr;
    OCI_CK(c0, db.alloc(&d_full, full.size()));
    size_t o = 0;
    for (Cls &q : cls) {
      q.d_all_full = d_full + o;
      o += q.qall.size();
      q.d_tiles_full = d_full + o;
      o += q.qtiles.size();
    }
    OCI_CK(c0, hipMemcpyAsync(d_full, full.data(), full.size() * sizeof(int2),
                              hipMemcpyHostToDevice, st));
    OCI_CK(c0, hipStreamSynchronize(st));   // (full is freed at the end of this block)
  }
  for (Cls &q : cls) {
    OCI_CK(c0, hipFuncSetAttribute((const void *)q.fb, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)q.lb));
    OCI_CK(c0, hipFuncSetAttribute((const void *)q.fi, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)q.li));
    OCI_CK(c0, hipFuncSetAttribute((const void *)q.fe, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)q.le));
  }
  std::vector<StepArgs> probs(n_ctx);
  std::vector<double *> phis(n_ctx, nullptr);
  for (int i = 0; i < n_ctx; ++i) {
    probs[i] = ctx[i]->sa;
    phis[i] = phi_out ? phi_out[i] : nullptr;
  }
  // the tables of a batch over a set of problems: the problem list, first,
  // last and, per class, the queues (every tile, and as "all" also each
  // problem's reduction work-group) -- for every problem the ones uploaded
  // above, for a subset its own
  std::vector<int> plist, first(n_ctx, 1), last(n_ctx, 1);
  auto build = [&](const std::vector<int> &set) -> int {
    const bool all = (int)set.size() == n_ctx;   // (sets are distinct indices)
    if (!all) {
      for (Cls &q : cls) {
        q.qall.clear();
        q.qtiles.clear();
      }
      for (int i : set) {
        Cls &q = cls[cls_of[i]];
        for (int t = 0; t <= ctx[i]->ntiles; ++t) q.qall.push_back(make_int2(i, t));
        for (int t = 0; t < ctx[i]->ntiles; ++t) q.qtiles.push_back(make_int2(i, t));
      }
    }
    plist = set;
    for (Cls &q : cls) q.L = 0;
    for (int i : set) {   // the class's launches: nodes 1 .. L
      Cls &q = cls[cls_of[i]];
      q.L = std::max(q.L, last[i] - first[i] + 1);
    }
    size_t off = 0;
    bool over = false;
    auto put = [&](const void *src, size_t n) {   // n ints at the next even offset
      if (off + n > pack_cap) {
        over = true;
        return d_pack;
      }
      std::memcpy(h_pack + off, src, n * sizeof(int));
      const size_t at = off;
      off += (n + 1) & ~(size_t)1;
      return d_pack + at;
    };
    d_plist = put(plist.data(), plist.size());
    d_first = put(first.data(), n_ctx);
    d_last = put(last.data(), n_ctx);
    for (Cls &q : cls) {
      if (all) {
        q.na = (size_t)q.nt_all;
        q.nt = (size_t)q.nt_tiles;
        q.d_qall = q.d_all_full;
        q.d_qtiles = q.d_tiles_full;
      } else {
        q.na = q.qall.size();
        q.nt = q.qtiles.size();
        q.d_qall = reinterpret_cast<int2 *>(put(q.qall.data(), 2 * q.qall.size()));
        q.d_qtiles = reinterpret_cast<int2 *>(put(q.qtiles.data(), 2 * q.qtiles.size()));
      }
    }
    if (over) return fail(c0, OCI_EDEVICE, "ensemble tables exceed their buffer");
    OCI_CK(c0, hipMemcpyAsync(d_pack, h_pack, off * sizeof(int), hipMemcpyHostToDevice, st));
    return OCI_OK;
  };
  OCI_CK(c0, hipMemcpyAsync(d_probs, probs.data(), n_ctx * sizeof(StepArgs),
                            hipMemcpyHostToDevice, st));
  OCI_CK(c0, hipMemcpyAsync(d_phis, phis.data(), n_ctx * sizeof(double *),
                            hipMemcpyHostToDevice, st));
  OCI_CK(c0, hipMemcpyAsync(d_ki, kin.data(), n_ctx * sizeof(int), hipMemcpyHostToDevice, st));
  std::vector<int> everyone(n_ctx);
  for (int i = 0; i < n_ctx; ++i) everyone[i] = i;
  // control-block writes for the problems of the current tables (d_plist)
  auto set_ctl = [&](int n, int psi_base) -> int {
    void *cargs[] = {&d_probs, &d_plist, &n, &psi_base};
    OCI_CK(c0, hipLaunchKernel((const void *)kb_set_ctl, dim3((unsigned)((n + 255) / 256)),
                               dim3(256), cargs, 0, st));
    return OCI_OK;
  };
  int worst = OCI_OK;
  int half = c0->parity;
  const dim3 blk(256);
  // launches over the current queues, one per class present
  auto begin = [&]() -> int {
    for (Cls &q : cls) {
      if (q.nt == 0) continue;
      void *bargs[] = {&d_probs, &q.d_qtiles};
      OCI_CK(c0, hipLaunchKernel((const void *)q.fb, dim3((unsigned)q.nt), q.bb, bargs,
                                 q.lb, st));
    }
    return OCI_OK;
  };
  // (a class of KI iterates per launch launches at nodes 1, 1 + KI, ...)
  auto iterate = [&](int node) -> int {
    for (Cls &q : cls) {
      if (q.na == 0 || node > q.L || !ocip::ens_launch_node(node, q.KI)) continue;
      void *args[] = {&d_probs, &q.d_qall, &d_first, &d_last, &node, &half};
      OCI_CK(c0, hipLaunchKernel((const void *)q.fi, dim3((unsigned)q.na), q.bi, args,
                                 q.li, st));
    }
    return OCI_OK;
  };
  auto finish = [&]() -> int {
    void *rargs[] = {&d_probs, &d_plist, &d_first, &d_last, &d_ki, &half};
    OCI_CK(c0, hipLaunchKernel((const void *)kb_reduce_rec, dim3((unsigned)plist.size()), blk,
                               rargs, 0, st));
    double **ph = phi_out ? d_phis : nullptr;
    int mode = 1 | (1 << 1);   // records reduced before; one trailing iterate
    for (Cls &q : cls) {
      if (q.nt == 0) continue;
      void *eargs[] = {&d_probs, &ph, &q.d_qtiles, &d_first, &d_last, &half, &mode};
      OCI_CK(c0, hipLaunchKernel((const void *)q.fe, dim3((unsigned)q.nt), q.be, eargs,
                                 q.le, st));
    }
    return OCI_OK;
  };
  for (int s = 0; s < n_steps; ++s) {
    // each problem's planned iterates: its count of the previous step
    bool need_begin = false;
    int L = 1;
    for (int i = 0; i < n_ctx; ++i) {
      need_begin |= !ctx[i]->gh_valid;
      const int want = ctx[i]->batch_hint > 0 ? ctx[i]->batch_hint : kColdBatch;
      first[i] = 1;
      last[i] = std::max(1, std::min({want, cap, ctx[i]->max_iters}));
      L = std::max(L, last[i]);
    }
    int rc = build(everyone);
    if (rc == OCI_OK && s == 0) rc = set_ctl(n_ctx, c0->parity);   // the solve opens
    if (rc) return rc;
    OCI_CK(c0, hipEventRecord(c0->ev0, st));
    if (need_begin) {
      rc = begin();
      if (rc) return rc;
      for (int i = 0; i < n_ctx; ++i) ctx[i]->gh_valid = true;
    }
    for (int l = 1; l <= L && rc == OCI_OK; ++l) rc = iterate(l);
    if (rc == OCI_OK) rc = finish();
    if (rc) return rc;
    OCI_CK(c0, hipStreamSynchronize(st));
    // problems still undecided: further single-iterate launches over them alone
    std::vector<int> open;
    for (int i = 0; i < n_ctx; ++i) {
      const int stt = ctx[i]->h_rec[s].status;
      if (stt == kNonFinite) return abandon_step(ctx[i], infos && infos[i] ? &infos[i][s] : nullptr,
                                                 ctx[i]->h_rec[s].accepted);
      if (stt == kRunning) open.push_back(i);
    }
    // undecided problems (each ran its planned iterates 1 .. last[i]) go on
    // from there, in batches of 1, 1, 2, 4, ... iterates (as a resumed step)
    int extra = 0;
    while (!open.empty()) {
      ++extra;
      int count = 1;
      for (int i : open) {
        ctx[i]->h_ctl->stalled = 0;   // (the device copies: kb_set_ctl after the tables)
        const int n = ocip::resumed_batch(extra, last[i], ctx[i]->max_iters, ctx[i]->nbuf);
        first[i] = last[i] + 1;
        last[i] += n;
        count = std::max(count, n);
      }
      rc = build(open);
      if (rc == OCI_OK) rc = set_ctl((int)open.size(), -1);
      for (int l = 1; l <= count && rc == OCI_OK; ++l) rc = iterate(l);
      if (rc == OCI_OK) rc = finish();
      if (rc) return rc;
      OCI_CK(c0, hipStreamSynchronize(st));
      std::vector<int> still;
      for (int i : open) {
        const int stt = ctx[i]->h_rec[s].status;
        if (stt == kNonFinite)
          return abandon_step(ctx[i], infos && infos[i] ? &infos[i][s] : nullptr,
                              ctx[i]->h_rec[s].accepted);
        if (stt == kRunning) still.push_back(i);
      }
      open.swap(still);
      for (int i : open)
        if (last[i] > ctx[i]->max_iters + 1)
          return fail(c0, OCI_EDEVICE, "an ensemble step did not reach a decision");
    }
    OCI_CK(c0, hipEventRecord(c0->ev1, st));
    OCI_CK(c0, hipEventSynchronize(c0->ev1));
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, c0->ev0, c0->ev1);
    for (int i = 0; i < n_ctx; ++i) {
      oci_ctx *c = ctx[i];
      const StepRecord &r = c->h_rec[s];
      const int status = r.status == kConverged ? OCI_OK : OCI_NOT_CONVERGED;
      if (status == OCI_NOT_CONVERGED) worst = OCI_NOT_CONVERGED;
      fill_info(infos && infos[i] ? &infos[i][s] : nullptr, r.accepted, status, r.e_last, ms, ms,
                r.accepted, error_bound(r.e_last, r.e_prev));
      complete_step(c, r.accepted);
      c->batch_hint = std::max(r.accepted, 1);
      c->window = 1;
    }
    half ^= 1;
  }
  return worst;
}

extern "C" int oci_get_flux(oci_ctx *c, double *phi, int32_t on_device) {
  if (!c || !phi) return fail(c, OCI_EINVAL, "NULL argument");
  if (!c->have_flux) return fail(c, OCI_ESTATE, "no step has completed yet");
  OCI_CK(c, hipMemcpyAsync(phi, c->d_phi_res, (size_t)c->J * 4 * sizeof(double),
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
  OCI_CK(c, hipStreamSynchronize(c->stream));
  return OCI_OK;
}

extern "C" int oci_get_state(oci_ctx *c, double *psi_edge, int64_t *step) {
  if (!c) return fail(nullptr, OCI_EINVAL, "context is NULL");
  if (psi_edge) {
    OCI_CK(c, hipMemcpyAsync(psi_edge, c->d_psi[c->parity], (size_t)c->J * 2 * c->N * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream));
    OCI_CK(c, hipStreamSynchronize(c->stream));
  }
  if (step) *step = c->steps;
  return OCI_OK;
}

extern "C" int oci_set_state(oci_ctx *c, const double *psi_edge, int64_t step) {
  if (!c) return fail(nullptr, OCI_EINVAL, "context is NULL");
  if (step < 0) return fail(c, OCI_EINVAL, "step must be >= 0");
  const size_t cnt = (size_t)c->J * 2 * c->N;
  if (psi_edge) {
    for (size_t i = 0; i < cnt; ++i)
      if (!std::isfinite(psi_edge[i])) return fail(c, OCI_EINVAL, "psi_edge must be finite");
  }
  int rc = reset_iterate(c, psi_edge == nullptr);   // (psi = 0 with the reset)
  if (rc) return rc;
  c->parity = 0;
  if (psi_edge) {   // read before the call returns
    OCI_CK(c, hipMemcpyAsync(c->d_psi[0], psi_edge, cnt * sizeof(double), hipMemcpyHostToDevice,
                             c->stream));
    OCI_CK(c, hipStreamSynchronize(c->stream));
  }
  c->steps = step;
  c->have_flux = false;
  return OCI_OK;
}

extern "C" int oci_get_quadrature(const oci_ctx *c, double *mu, double *w) {
  if (!c) return fail(nullptr, OCI_EINVAL, "context is NULL");
  if (mu) std::copy(c->mu.begin(), c->mu.end(), mu);
  if (w) std::copy(c->w.begin(), c->w.end(), w);
  return OCI_OK;
}

extern "C" int oci_get_sizes(const oci_ctx *c, int32_t *n_angles, int32_t *n_cells,
                             int32_t *n_regions) {
  if (!c) return fail(nullptr, OCI_EINVAL, "context is NULL");
  if (n_angles) *n_angles = c->N;
  if (n_cells) *n_cells = c->J;
  if (n_regions) *n_regions = c->R;
  return OCI_OK;
}

extern "C" int oci_iterates_per_launch(const oci_ctx *c) {
  if (!c) return fail(nullptr, OCI_EINVAL, "context is NULL");
  return c->mixed ? 1 : c->kimax;
}

extern "C" int oci_set_iterates_per_launch(oci_ctx *c, int32_t k) {
  if (!c) return fail(nullptr, OCI_EINVAL, "context is NULL");
  if (k < 1) return fail(c, OCI_EINVAL, "iterates per launch must be >= 1");
  if (c->mixed) return 1;
  const int v = std::min<int>(k, c->kibuilt);
  if (v != c->kimax) {
    drop_step_graphs(c);   // the cached step graphs hold the old launch sequence
    c->kimax = v;
  }
  return v;
}

extern "C" int oci_end_fusion(const oci_ctx *c) {
  if (!c) return fail(nullptr, OCI_EINVAL, "context is NULL");
  return c->fuse_end ? 1 : 0;
}

extern "C" int oci_set_end_fusion(oci_ctx *c, int32_t on) {
  if (!c) return fail(nullptr, OCI_EINVAL, "context is NULL");
  const bool v = on != 0;
  if (v != c->fuse_end) drop_step_graphs(c);   // cached graphs hold the old sequence
  c->fuse_end = v;
  return v ? 1 : 0;
}

extern "C" int oci_inner_iterations(const oci_ctx *c) {
  if (!c) return fail(nullptr, OCI_EINVAL, "context is NULL");
  return c->mixed ? c->m_inner : 0;
}

extern "C" int oci_set_inner_iterations(oci_ctx *c, int32_t m) {
  if (!c) return fail(nullptr, OCI_EINVAL, "context is NULL");
  if (m < 0 || m > kMaxInner) return fail(c, OCI_EINVAL, "inner iterations must be in [0, 64]");
  if (!c->mixed) return 0;
  const int v = m == 0 ? c->m_inner : m;
  if (v != c->m_inner) drop_step_graphs(c);   // cached graphs hold the old sequence
  c->m_inner = v;
  c->m_fixed = m != 0;
  c->m_q = c->m_prev = c->m_prev_q = 0;
  c->m_locked = false;
  return v;
}

extern "C" int oci_get_operator(oci_ctx *c, int32_t region, double *op) {
  if (!c || !op) return fail(c, OCI_EINVAL, "NULL argument");
  if (region < 0 || region >= c->R) return fail(c, OCI_EINVAL, "region out of range");
  const size_t per = (size_t)(4 * c->N + 4) * (4 * c->N + 1);
  OCI_CK(c, hipMemcpyAsync(op, c->d_op + region * per, per * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
  OCI_CK(c, hipStreamSynchronize(c->stream));
  return OCI_OK;
}

extern "C" void oci_destroy(oci_ctx *c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  drop_graphs(c);
  for (void *q : c->allocs) (void)hipFree(q);
  if (c->h_ctl) (void)hipHostFree(c->h_ctl);
  if (c->h_rec) (void)hipHostFree(c->h_rec);
  if (c->h_dec) (void)hipHostFree(c->h_dec);
  for (hipEvent_t e : {c->ev0, c->ev1, c->evA, c->evB, c->evW[0][0], c->evW[0][1], c->evW[1][0],
                       c->evW[1][1]})
    if (e) (void)hipEventDestroy(e);
  delete c;
}

extern "C" const char *oci_strerror(int code) {
  switch (code) {
    case OCI_OK: return "ok";
    case OCI_NOT_CONVERGED: return "iteration limit reached before the stopping rule";
    case OCI_EINVAL: return "invalid argument";
    case OCI_ENOMEM: return "device memory allocation failed";
    case OCI_EDEVICE: return "HIP runtime error";
    case OCI_ENONFINITE: return "scalar flux became NaN or Inf";
    case OCI_ESTATE: return "call not valid in the current state";
    default: return "unknown error code";
  }
}

extern "C" const char *oci_last_error(const oci_ctx *c) {
  if (c) return c->err.c_str();
  return g_last_error.c_str();
}
