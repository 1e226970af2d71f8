// Kernel argument blocks and kernel declarations shared by the host driver
// (api.hip) and the kernel translation units.
#pragma once

#include "oci_device.h"

namespace ocik {

// Tiles whose descriptors travel in the kernel arguments (one scalar load
// with the other arguments, no dependent table load on the launch's critical
// path); larger problems read the TileDev table.  A descriptor word packs
// c0 (bits 0-17), nc - 1 (bits 18-21) and the region (bits 22-31).
constexpr int kArgTiles = 768;
constexpr int kArgTileCellBits = 18;
__host__ __device__ inline uint32_t pack_tile(int region, int c0, int nc) {
  return (uint32_t)c0 | ((uint32_t)(nc - 1) << kArgTileCellBits) | ((uint32_t)region << 22);
}
// Per (region, angle) coefficients of the structured apply (see oci_step.hip).
constexpr int kCoef = 36;
// Iterate buffers per ring half at most (iterate ranges of one end of step
// span fewer).
constexpr int kMaxRing = 65;
constexpr int kMaxTrail = 4;   // most iterates per launch (the end reduces theirs)
// LDS rows of the two-iterate kernel: iterate l-1 of cells c0-2 .. c0+17,
// iterate l of cells c0-1 .. c0+16.
constexpr int kBlkA = 16 + 4, kBlkB = 16 + 2;

struct StepArgs {
  const TileDev *tiles;    // [ntiles] in work-group order (one work-group per tile)
  int ntiles;
  int tiles_in_args;       // 1: tile_word holds every tile's descriptor (kernels <.., true>)
  uint32_t tile_word[kArgTiles]; // packed descriptors in work-group order (see pack_tile)
  int N, J, Mt, Met;
  int Mto;                 // row tiles holding the 2N outgoing rows
  int R;                   // regions
  int bcl, bcr;
  int max_iters, strict;
  double tol;
  const double *frag_it;   // G (iteration), per region stride frag_it_stride
  size_t frag_it_stride;
  const double *frag_pv;   // P (per-step constant)
  size_t frag_pv_stride;
  const double *c_pv;      // p
  size_t c_pv_stride;
  const RegionDev *regions; // [R] cell width and cross sections (end of step)
  const double *mu;        // [N]
  const double *ainv;      // [R][N][16] A_m^{-1} per region and angle
  const double *coef;      // [R][kCoef/2][N][2] outgoing-pair and step-constant coefficients
                           //   (pairs of coefficients, pair-major: see write_out_coef)
  const double *phig;      // [R][4][2N] scalar-flux rows of G (incident columns), plain
  const int *cell_region;  // [J] (halo cells of the two-iterate kernel)
  double at;               // 1/(v dt), 0 for v = inf
  double *gh;              // [J][Mt*16]
  int nbuf;                // ring slots per half (iterate l of a step in slot l % nbuf)
  double *outb;            // [2*nbuf+2][J+2][2N]
  size_t out_stride;
  double *phib;            // [2*nbuf+2][J][4]
  size_t phi_stride;
  double *psi0, *psi1;     // [J][2N]
  double *phi_res;         // [J][4]
  double *partial;         // [2][nbuf][ntiles] double2 residual records: iterate l of a step
                           //   of ring half h in slot h*nbuf + l % nbuf
  double *dec;             // [nbuf] e of iterate l in slot l % nbuf (NaN: not finite)
  StepCtl *ctl;
  StepRecord *rec;         // [steps] records of a queued solve
  // mixed precision (FP64 defect correction with FP32 inner iterations)
  const float *frag_it32;  // G in FP32, same packing and stride as frag_it
  float *dlt;              // [3][J+2][2N] FP32: the defect d (buffer 0) and the inner
  size_t dlt_stride;       //   iterates (1, 2); ghost rows zero
  float *dphi32;           // [J][4] FP32 scalar-flux part of the defect
};

// Affine map of a sweep's (level k, level k+1/2) flux pair: x -> M x + v.
struct Affine {
  double m00, m01, m10, m11, v0, v1;
};

struct SiArgs {
  int N, J, bcl, bcr, max_iters, strict;
  double tol, a;
  const RegionDev *regions;
  const int *cell_region;   // [J]
  const double *mu, *w;
  const double *ainv;       // [R][N][16]
  double *out0, *out1;      // [J+2][2N] iterate buffers own_buf and own_buf+1 (ghost rows
  double *phi0, *phi1;      //   hold incident values); [J][4]
  int own_buf;
  double *outb;             // all iterate buffers (as StepArgs): the step start moves the
  size_t out_stride;        //   previous step's last iterate from buffer fin_buf to own_buf
  double *phib;
  size_t phi_stride;
  double *psi0, *psi1;      // [J][2N]
  double *contrib;          // [ncontrib][J][4] partial sums of w_m psi_m (angle-pair
                            //   sweep: one per pair; angle-lane sweep: one per direction)
  int ncontrib;
  double *lag;              // [2][N/2][2] right-edge outgoing flux of the mu > 0 angle,
                            //   by iterate parity (both edges reflecting)
  Affine *segmap;           // [N/2][S][2] segment maps of the two sweep directions
                            //   (angle-lane sweep: [2][nseg][N/2])
  double2 *segin;           // angle-lane sweep: [2][nseg][N/2] flux entering each segment
  Affine *chmap;            // angle-lane sweep: [2][nseg][256] chunk maps, by thread
  int nseg;                 // angle-lane sweep: segments
  double *phi_res;          // [J][4]
  double *partial;          // [3][nparts] double2 residual records
  int nparts;
  StepCtl *ctl;
};

// Ranges of doubles to clear in one launch (k_zero).
struct ZeroRanges {
  double *p[6];
  size_t n[6];
  int count;
};

// Operator tables of a solve (k_region_setup).
struct SetupArgs {
  const RegionDev *regions;  // [R]
  const double *mu, *w;      // [N]
  int N, Mt;
  double a;                  // 1/(v dt), 0 for v = inf
  double *ainv;              // [R][N][16] A_m^{-1}
  double *coef;              // [R][kCoef/2][N][2]
  double *phig;              // [R][4][2N]
  double *op;                // [R][4N+4][4N+1] operator rows
  double *frag_it, *frag_pv; // G and P in fragment order, per region stride frag_stride
  float *frag_it32;          // G in FP32 (mixed precision), or null
  size_t frag_stride;
  double *c_pv;              // p, per region stride cvec_stride
  size_t cvec_stride;
  int *bad;                  // set to 1 when a region's 4x4 system is singular
};

// setup.hip
__global__ void k_zero(ZeroRanges z);
__global__ void k_region_setup(SetupArgs q);
// oci_step.hip (CH = operator k-steps fetched per batch: 4, 8 or 16)
// ARGT: tile descriptors in the kernel arguments; VEC: 16-byte operand
// reads (N % 8 == 0); NF > 0: built for N = NF angles, 0: any N.
template <int CH, bool ARGT, bool VEC, int NF> __global__ void k_step_begin(StepArgs a);
// half: the ring half of the step's iterates.  rmode bits 0-1 (rstep): 1 for
// plain FP64 OCI; 2 for the mixed-precision step, where the FP64 iterates are
// every other one (iterate l even is formed by the FP32 inner iterations) and
// each FP64 iterate also writes its defect in FP32; bit 2: the outgoing
// fluxes are not stored, bit 3: the defect is not stored.  nred: iterates of
// the previous launch whose residual this launch reduces (2 after a
// two-iterate launch).
template <int CH, bool ARGT, bool VEC, int NF>
__global__ void k_oci_iterate(StepArgs a, int node, int cb, int half, int rmode, int nred);
// The FP32 defect of FP64 iterate l against its starting point (mixed
// precision, resumed steps).
__global__ void k_defect(StepArgs a, int l, int half);
// Iterates l = cb + node and l + 1 in one launch (plain FP64 OCI); nred: the
// previous launch's iterates, whose residuals the extra work-group reduces.
template <int CH, bool ARGT, bool VEC, int NF>
__global__ void k_oci_iterate2(StepArgs a, int node, int cb, int half, int nred);
// Iterates l .. l+KI-1 in one launch (KI = 3, 4; built for N = 8, 16, 32, 64).
template <int CH, bool ARGT, bool VEC, int NF, int KI>
__global__ void k_oci_iterateK(StepArgs a, int node, int cb, int half, int nred);
// mode bit 0: the e of the trailing iterates are already in dec (k_reduce_rec
// ran before); bits 1-3: the trailing iterates (those of the batch's last
// launch, 1 .. 4), whose e this kernel forms; bit 4: a decided step also
// computes iterate 1 of the next step (plain OCI; the next step's launches
// start at 2); bit 5: that iterate (mixed precision, a correction follows)
// does not store its outgoing fluxes.
template <int CH, bool ARGT, bool VEC, int NF>
__global__ void k_step_end(StepArgs a, double *phi_out, int first, int last, int half,
                           int rstep, int mode);
// The same without the fused iterate (bit 4 ignored; fewer registers).
template <int CH, bool ARGT, bool VEC, int NF>
__global__ void k_step_end_nf(StepArgs a, double *phi_out, int first, int last, int half,
                              int rstep, int mode);
// e of iterates l-n+1 .. l from their residual records into dec, one
// work-group per iterate (grid n).
__global__ void k_reduce_rec(StepArgs a, int l, int n, int half);
// FP32 inner iteration i (1-based) of a mixed-precision step; ly > 0: the last
// one, which also forms FP64 iterate ly (the point iterate ly-1 started from
// plus the correction); opens: the step's first launch (its FP64 iterate 1
// came with the previous end of step).
template <bool ARGT>
__global__ void k_oci_inner(StepArgs a, int i, int ly, int half, int opens);
// Two inner iterations in one launch (halo cells recomputed); n: the launch's
// index within the correction (selects the buffers as i does above).
template <bool ARGT>
__global__ void k_oci_inner2(StepArgs a, int n, int ly, int half, int opens);
// Ensembles: the same step kernels (NF: built for N = NF with that N's work-group
// size, or 0: any N, a multiple of 8, 256 threads) over
// a work queue of (problem, tile) entries, each problem with its own argument
// block probs[problem]; a tile entry equal to the problem's tile count is its
// residual-reduction work-group (kb_oci_iterate).  first[problem] ..
// last[problem]: the iterates of the current batch of that problem (launch
// `node` computes iterate first + node - 1; launches past last leave it idle;
// the end of step judges first .. last).  kb_oci_iterateK: launch `node`
// (1, 1 + KI, 1 + 2 KI, ...) computes the problem's iterates first + node - 1
// .. of at most KI, up to last.  kb_reduce_rec: one work-group per problem of
// plist, reducing the iterates of its last launch (ki[problem] iterates per
// launch).  kb_step_end: phi_outs[problem] (or NULL) receives the accepted
// scalar flux as phi_out does in k_step_end (rstep 1).
template <int CH, int NF> __global__ void kb_step_begin(const StepArgs *probs, const int2 *queue);
template <int CH, int NF>
__global__ void kb_oci_iterate(const StepArgs *probs, const int2 *queue, const int *first,
                               const int *last, int node, int half);
template <int CH, int NF, int KI>
__global__ void kb_oci_iterateK(const StepArgs *probs, const int2 *queue, const int *first,
                                const int *last, int node, int half);
__global__ void kb_reduce_rec(const StepArgs *probs, const int *plist, const int *first,
                              const int *last, const int *ki, int half);
template <int CH, int NF>
__global__ void kb_step_end(const StepArgs *probs, double *const *phi_outs, const int2 *queue,
                            const int *first, const int *last, int half, int mode);
// The control blocks of the problems plist[0 .. n-1], one thread each:
// psi_base >= 0 opens a solve (next step 0, psi_{k-1/2} of step 0 in buffer
// psi_base), psi_base < 0 clears the stall flag before a resumed batch.
__global__ void kb_set_ctl(const StepArgs *probs, const int *plist, int n, int psi_base);
// Learned corrections of iterate l of the open step (ring half `half`): the
// corrector's FP32 input (ch = 8 or 12 channels; amp: the extrapolation
// factor of channels 8..11) from the scalar fluxes of iterates l-2 .. l, and
// the corrected iterate in place from its output y [4][J].
__global__ void k_learn_features(StepArgs a, int l, int half, int ch, double amp, float *x);
__global__ void k_learn_apply(StepArgs a, int l, int half, const float *y);
// si.hip
__global__ void k_si_maps(SiArgs a, int node, int cb);
// The angle-lane sweep (N/2 a power of two, N <= 128): grid (nseg, 2) for the
// segment maps and the sweep, grid N/2 for the segments' entering fluxes.
__global__ void k_si_smaps(SiArgs a, int node, int cb);
__global__ void k_si_enter(SiArgs a, int node, int cb);
__global__ void k_si_lsweep(SiArgs a, int node, int cb);
__global__ void k_si_sweep(SiArgs a, int node, int cb);
__global__ void k_si_reduce(SiArgs a, int node, int cb);
__global__ void k_si_decide(SiArgs a, int node, int cb);
__global__ void k_si_begin(SiArgs a, int parity);
__global__ void k_si_end(SiArgs a);

}  // namespace ocik
