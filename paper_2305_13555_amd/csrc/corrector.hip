// Learned iterate corrector: a small 1-D convolutional network over cells,
// trained on OCI iterate histories that the solver generates, to damp the
// slow convergence of OCI in optically thin cells (the weakness the paper
// states in its introduction and conclusions; the paper has no corrector).
//
// Network: four convolutions over cells (kernel width 5, two cells of zero
// padding at each mesh end), 32 channels between layers, no biases, ReLU
// after the first three.  Without biases the network is positively
// homogeneous, f(a x) = a f(x) for a > 0, so a predicted correction scales
// with the iterate differences it is fed.  Training: mean squared error,
// Adam (Kingma and Ba, 2015).  FP64 throughout.
//
// Layout: activations [B][C][J] (cells contiguous: a work-group's threads
// read consecutive cells); weights of layer l [C_o][C_i][5], layers
// concatenated.  The work is small next to an OCI iterate of the same mesh
// and bound by latency; the kernels are plain and coalesced.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "oci.h"
#include "corrector_internal.h"

namespace occ {

constexpr int KW = 5, HID = 32, NL = 4, COT = 4;

// y[b][o][j] = sum_i sum_t W[o][i][t] x[b][i][j + t - 2] (zero outside the
// mesh), ReLU if relu.  Grid (ceil(J/256), Co/CT, B); CT outputs per thread
// (8 where Co allows: fewer re-reads of x per output).  The work-group's 260
// input cells are staged in LDS kStageCh channels at a time, so each x value
// is read from memory once per work-group instead of once per tap.
constexpr int kStageCh = 8, kSpan = 256 + KW - 1;
template <int CT>
__global__ __launch_bounds__(256) void k_conv_fwd(const double *__restrict__ x, int Ci, int J,
                                                  const double *__restrict__ W, int Co,
                                                  double *__restrict__ y, int relu) {
  __shared__ double xs[kStageCh][kSpan];
  const int j0 = blockIdx.x * 256, j = j0 + threadIdx.x;
  const int o0 = blockIdx.y * CT, b = blockIdx.z;
  double acc[CT];
#pragma unroll
  for (int o = 0; o < CT; ++o) acc[o] = 0.0;
  const double *xb = x + (size_t)b * Ci * J;
  for (int i0 = 0; i0 < Ci; i0 += kStageCh) {
    const int nc = min(kStageCh, Ci - i0);
    __syncthreads();   // the previous channels' reads are done
    for (int e = threadIdx.x; e < nc * kSpan; e += blockDim.x) {
      const int ii = e / kSpan, c = e - ii * kSpan, k = j0 - 2 + c;
      xs[ii][c] = (k >= 0 && k < J) ? xb[(size_t)(i0 + ii) * J + k] : 0.0;
    }
    __syncthreads();
    for (int ii = 0; ii < nc; ++ii) {
      double xv[KW];
#pragma unroll
      for (int t = 0; t < KW; ++t) xv[t] = xs[ii][threadIdx.x + t];   // x[j + t - 2]
#pragma unroll
      for (int o = 0; o < CT; ++o)
#pragma unroll
        for (int t = 0; t < KW; ++t) acc[o] += W[((size_t)(o0 + o) * Ci + i0 + ii) * KW + t] * xv[t];
    }
  }
  if (j >= J) return;
#pragma unroll
  for (int o = 0; o < CT; ++o)
    y[((size_t)b * Co + o0 + o) * J + j] = relu ? fmax(acc[o], 0.0) : acc[o];
}

// Gradient wrt a layer's input: gx[b][i][k] = sum_o sum_t W[o][i][t]
// g[b][o][k - t + 2], times the ReLU mask of that input (act > 0) when act is
// given (the input is the previous layer's ReLU output).  Grid (ceil(J/256),
// Ci/CT, B).
template <int CT>
__global__ __launch_bounds__(256) void k_conv_bwd_data(const double *__restrict__ g, int Co, int J,
                                                       const double *__restrict__ W, int Ci,
                                                       const double *__restrict__ act,
                                                       double *__restrict__ gx) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int i0 = blockIdx.y * CT, b = blockIdx.z;
  if (k >= J) return;
  double acc[CT];
#pragma unroll
  for (int i = 0; i < CT; ++i) acc[i] = 0.0;
  const double *gb = g + (size_t)b * Co * J;
  for (int o = 0; o < Co; ++o) {
    double gv[KW];
#pragma unroll
    for (int t = 0; t < KW; ++t) {
      const int j = k - t + 2;
      gv[t] = (j >= 0 && j < J) ? gb[(size_t)o * J + j] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < CT; ++i)
#pragma unroll
      for (int t = 0; t < KW; ++t) acc[i] += W[((size_t)o * Ci + i0 + i) * KW + t] * gv[t];
  }
#pragma unroll
  for (int i = 0; i < CT; ++i) {
    const size_t e = ((size_t)b * Ci + i0 + i) * J + k;
    gx[e] = (act && !(act[e] > 0.0)) ? 0.0 : acc[i];
  }
}

// Block sum of 256 threads' values (deterministic order).
__device__ inline double block_sum(double v, double *sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) sh[tid] += sh[tid + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Weight gradient: dW[o][i][t] = sum_b sum_j g[b][o][j] x[b][i][j + t - 2].
// Layers wider than kTileCh channels: one work-group of 256 per (o, i) (grid
// Co x Ci), the threads striding over (b, j), then the work-group sums each
// tap (every work-group re-reads its two rows; the tiled form below reads
// each row once per pair group).
__global__ __launch_bounds__(256) void k_conv_bwd_weight(const double *__restrict__ g, int Co,
                                                         const double *__restrict__ x, int Ci,
                                                         int J, int B, double *__restrict__ dW) {
  __shared__ double sh[256];
  const int o = blockIdx.x, i = blockIdx.y;
  double acc[KW];
#pragma unroll
  for (int t = 0; t < KW; ++t) acc[t] = 0.0;
  const size_t n = (size_t)B * J;
  for (size_t e = threadIdx.x; e < n; e += blockDim.x) {
    const int b = (int)(e / J), j = (int)(e - (size_t)b * J);
    const double gv = g[((size_t)b * Co + o) * J + j];
    const double *xr = x + ((size_t)b * Ci + i) * J;
#pragma unroll
    for (int t = 0; t < KW; ++t) {
      const int k = j + t - 2;
      acc[t] += (k >= 0 && k < J) ? gv * xr[k] : 0.0;
    }
  }
#pragma unroll
  for (int t = 0; t < KW; ++t) {
    const double s = block_sum(acc[t], sh);
    if (threadIdx.x == 0) dW[((size_t)o * Ci + i) * KW + t] = s;
  }
}

// Weight gradient for layers of at most kTileCh input and output channels,
// in two passes.  Pass 1, grid (nbx, ceil(Co*Ci / 1024)): work-group (bx, y)
// takes the chunks of kChunk cells bx, bx + nbx, ... of the batch, stages
// g[b][:][chunk] and x[b][:][chunk - 2 .. chunk + kChunk + 2) in LDS once,
// and each thread sums, for its (at most four) (o, i) pairs of pair group y,
// the five taps over the chunk; part[bx*n + (o*Ci + i)*KW + t] (n = Co*Ci*KW)
// holds the work-group's sums.  Pass 2 adds the nbx partial sums of every
// weight in order.  Dynamic LDS: (Co*kChunk + Ci*(kChunk+4)) doubles.
constexpr int kChunk = 32, kTileCh = 64, kPairs = 4;
__global__ __launch_bounds__(256) void k_conv_bwd_weight_part(const double *__restrict__ g, int Co,
                                                              const double *__restrict__ x, int Ci,
                                                              int J, int B,
                                                              double *__restrict__ part) {
  extern __shared__ double sh[];
  double *gs = sh;                   // [Co][kChunk]
  double *xs = sh + Co * kChunk;     // [Ci][kChunk + 4]
  const int nbx = gridDim.x, bx = blockIdx.x, tid = threadIdx.x;
  const int npair = Co * Ci, p0 = blockIdx.y * 256 * kPairs;
  const int nch = (J + kChunk - 1) / kChunk;
  double acc[kPairs][KW];
#pragma unroll
  for (int q = 0; q < kPairs; ++q)
#pragma unroll
    for (int t = 0; t < KW; ++t) acc[q][t] = 0.0;
  for (int c = bx; c < B * nch; c += nbx) {
    const int b = c / nch, j0 = (c - b * nch) * kChunk;
    __syncthreads();   // the previous chunk's reads are done
    for (int e = tid; e < Co * kChunk; e += blockDim.x) {
      const int o = e / kChunk, j = j0 + e % kChunk;
      gs[e] = j < J ? g[((size_t)b * Co + o) * J + j] : 0.0;
    }
    for (int e = tid; e < Ci * (kChunk + 4); e += blockDim.x) {
      const int i = e / (kChunk + 4), k = j0 - 2 + e % (kChunk + 4);
      xs[e] = (k >= 0 && k < J) ? x[((size_t)b * Ci + i) * J + k] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPairs; ++q) {
      const int p = p0 + q * 256 + tid;
      if (p < npair) {
        const double *gr = gs + (p / Ci) * kChunk;
        const double *xr = xs + (p % Ci) * (kChunk + 4);
#pragma unroll
        for (int j = 0; j < kChunk; ++j) {   // (unrolled: each x value serves five taps)
          const double gv = gr[j];
#pragma unroll
          for (int t = 0; t < KW; ++t) acc[q][t] += gv * xr[j + t];
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kPairs; ++q) {
    const int p = p0 + q * 256 + tid;
    if (p < npair)
#pragma unroll
      for (int t = 0; t < KW; ++t) part[(size_t)bx * npair * KW + (size_t)p * KW + t] = acc[q][t];
  }
}

// (eight running sums per weight, partials b = r, r + 8, ..., then added in
// order: eight loads in flight instead of one)
__global__ __launch_bounds__(64) void k_conv_bwd_weight_sum(const double *__restrict__ part,
                                                            int n, int nbx,
                                                            double *__restrict__ dW) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double s[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) s[r] = 0.0;
  int b = 0;
  for (; b + 8 <= nbx; b += 8)
#pragma unroll
    for (int r = 0; r < 8; ++r) s[r] += part[(size_t)(b + r) * n + e];
  for (int r = 0; b + r < nbx; ++r) s[r] += part[(size_t)(b + r) * n + e];
  double t = s[0];
#pragma unroll
  for (int r = 1; r < 8; ++r) t += s[r];
  dW[e] = t;
}

// Mean squared error: g = 2 (y - target) / n and per-work-group partial sums
// of (y - target)^2.
__global__ __launch_bounds__(256) void k_mse(const double *__restrict__ y,
                                             const double *__restrict__ target, size_t n,
                                             double *__restrict__ g, double *__restrict__ part) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const double d = y[e] - target[e];
    g[e] = 2.0 * d / (double)n;
    acc += d * d;
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// loss = sum of the partials / n (one work-group).
__global__ __launch_bounds__(256) void k_mse_finish(const double *__restrict__ part, int np,
                                                    size_t n, double *__restrict__ loss) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int e = threadIdx.x; e < np; e += blockDim.x) acc += part[e];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) *loss = s / (double)n;
}

// One Adam step; bc1 = 1 - beta1^t, bc2 = 1 - beta2^t (formed on the host).
__global__ __launch_bounds__(256) void k_adam(double *__restrict__ w, const double *__restrict__ g,
                                              double *__restrict__ m, double *__restrict__ v,
                                              size_t n, double lr, double b1, double b2,
                                              double eps, double bc1, double bc2) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const double ge = g[e];
    const double me = b1 * m[e] + (1.0 - b1) * ge;
    const double ve = b2 * v[e] + (1.0 - b2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    w[e] = w[e] - lr * (me / bc1) / (sqrt(ve / bc2) + eps);
  }
}

// FP32 copy of the weights for inference.
__global__ __launch_bounds__(256) void k_to_f32(const double *__restrict__ w, size_t n,
                                                float *__restrict__ w32) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    w32[e] = (float)w[e];
}

// Inference convolution in FP32 on the matrix cores: per work-group 64 cells
// (16 per wave) and every output channel, as the product
//   y[o][j] = sum_k W[o][k] X[k][j],  k = 5 i + t,  X[k][j] = x[i][j + t - 2]
// on v_mfma_f32_16x16x4f32 (A = W rows o, B = the shifted inputs of 16
// cells; lane l supplies A[l%16][l/16] and B[l/16][l%16] and receives
// D[4 (l/16) + r][l%16]).  The layer's weights (zero-padded to Co rounded up to
// 16 rows and Ci*5 rounded up to a multiple of 4) and the work-group's
// Ci x (64 + 4) input cells are staged in LDS.  Grid (ceil(J/64), 1, B);
// dynamic LDS: (MT*16*KP + Ci*(64+4)) floats, MT = ceil(Co/16), KP = Ci*5
// rounded up to 4.  Co <= 32.
constexpr int kC32 = 64;   // cells per work-group
__global__ __launch_bounds__(256) void k_conv_fwd32(const float *__restrict__ x, int Ci, int J,
                                                    const float *__restrict__ W, int Co,
                                                    float *__restrict__ y, int relu) {
  extern __shared__ float sm[];
  const int MT = (Co + 15) / 16, KP = (Ci * KW + 3) & ~3, XP = kC32 + KW - 1;
  float *ws = sm;                    // [MT*16][KP]
  float *xs = sm + MT * 16 * KP;     // [Ci][XP], column c <-> cell j0 - 2 + c
  const int j0 = blockIdx.x * kC32, b = blockIdx.z, tid = threadIdx.x;
  const float *xb = x + (size_t)b * Ci * J;
  for (int e = tid; e < MT * 16 * KP; e += blockDim.x) {
    const int o = e / KP, k = e - o * KP;
    ws[e] = (o < Co && k < Ci * KW) ? W[(size_t)o * Ci * KW + k] : 0.f;
  }
  for (int e = tid; e < Ci * XP; e += blockDim.x) {
    const int i = e / XP, c = e - i * XP, j = j0 - 2 + c;
    xs[e] = (j >= 0 && j < J) ? xb[(size_t)i * J + j] : 0.f;
  }
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63, col = lane & 15, kq = lane >> 4;
  typedef float f4v __attribute__((ext_vector_type(4)));
  f4v acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
  const int cw = wave * 16 + col;   // this lane's cell column within the work-group
  for (int ks = 0; ks < KP / 4; ++ks) {
    const int k = 4 * ks + kq;
    const int i = min(k / KW, Ci - 1), t = k - (k / KW) * KW;
    const float bv = xs[i * XP + cw + t];   // (k past Ci*5: the weights there are zero)
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
      if (mt < MT) acc[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ws[(mt * 16 + col) * KP + k], bv,
                                                                  acc[mt], 0, 0, 0);
  }
  const int j = j0 + cw;
  if (j >= J) return;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    if (mt >= MT) break;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int o = mt * 16 + 4 * kq + r;
      if (o < Co) {
        const float v = acc[mt][r];
        y[((size_t)b * Co + o) * J + j] = relu ? fmaxf(v, 0.f) : v;
      }
    }
  }
}

}  // namespace occ

using namespace occ;

struct oci_corrector {
  int c_in = 0, c_out = 0, max_batch = 0, max_cells = 0;
  hipStream_t stream = nullptr;
  std::string err;
  int chans[NL + 1] = {};
  size_t woff[NL + 1] = {};   // layer l's weights at w + woff[l]
  double *w = nullptr, *gw = nullptr, *m = nullptr, *v = nullptr;
  double *act[NL] = {};       // act[1..3]: hidden outputs; act[0] unused (the caller's x)
  double *y = nullptr;        // network output during training
  double *g0 = nullptr, *g1 = nullptr;   // gradient ping-pong [B][max(HID, c_out)][J]
  double *part = nullptr, *loss = nullptr;
  double *wpart = nullptr;    // weight-gradient partial sums [kWgtBlocks][Co*Ci*KW]
  int64_t adam_t = 0;
  float *w32 = nullptr;       // FP32 weights for inference (converted when stale)
  float *h32[2] = {};         // FP32 hidden activations, used in turn
  bool w32_stale = true;
};

namespace {

constexpr int kPartBlocks = 256;
constexpr int kWgtBlocks = 256;   // work-groups per pair group of the tiled weight gradient

int cfail(oci_corrector *k, int code, const std::string &msg) {
  if (k) k->err = msg;
  return code;
}

#define CK(k, call)                                                                  \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess) return cfail(k, OCI_EDEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

int check_shape(oci_corrector *k, int32_t batch, int32_t cells) {
  if (batch < 1 || cells < 1 || batch > k->max_batch || cells > k->max_cells)
    return cfail(k, OCI_EINVAL, "batch or cell count outside [1, maximum given at creation]");
  return OCI_OK;
}

// Forward pass of x [B][chans[0]][J] into out on stream st, weights w
// (layer l at w + woff[l]); the hidden outputs go to act[1..3].
hipError_t launch_forward(hipStream_t st, const double *w, const size_t *woff, const int *chans,
                          const double *x, int B, int J, double *out, double *const *act) {
  const double *in = x;
  for (int l = 0; l < NL; ++l) {
    const int Ci = chans[l], Co = chans[l + 1];
    double *o = l == NL - 1 ? out : act[l + 1];
    const double *W = w + woff[l];
    const int relu = l < NL - 1 ? 1 : 0;
    if (Co % 8 == 0)
      hipLaunchKernelGGL(k_conv_fwd<8>, dim3((J + 255) / 256, Co / 8, B), dim3(256), 0, st, in,
                         Ci, J, W, Co, o, relu);
    else
      hipLaunchKernelGGL(k_conv_fwd<COT>, dim3((J + 255) / 256, Co / COT, B), dim3(256), 0, st,
                         in, Ci, J, W, Co, o, relu);
    in = o;
  }
  return hipGetLastError();
}

// Forward pass of x [B][c_in][J] into out; hidden activations kept in act[1..3].
int forward(oci_corrector *k, const double *x, int B, int J, double *out) {
  CK(k, launch_forward(k->stream, k->w, k->woff, k->chans, x, B, J, out, k->act));
  return OCI_OK;
}

// Loss (on the device, k->loss) and every weight gradient (k->gw).
int gradient(oci_corrector *k, const double *x, const double *target, int B, int J) {
  int rc = forward(k, x, B, J, k->y);
  if (rc) return rc;
  const size_t n = (size_t)B * k->c_out * J;
  hipLaunchKernelGGL(k_mse, dim3(kPartBlocks), dim3(256), 0, k->stream, (const double *)k->y,
                     target, n, k->g0, k->part);
  hipLaunchKernelGGL(k_mse_finish, dim3(1), dim3(256), 0, k->stream, (const double *)k->part,
                     kPartBlocks, n, k->loss);
  double *g = k->g0, *gn = k->g1;
  for (int l = NL - 1; l >= 0; --l) {
    const int Ci = k->chans[l], Co = k->chans[l + 1];
    const double *in = l == 0 ? x : k->act[l];
    if (Co <= kTileCh && Ci <= kTileCh) {
      const int nch = B * ((J + kChunk - 1) / kChunk);
      const int nbx = std::min(kWgtBlocks, nch);
      const int ngrp = (Co * Ci + 256 * kPairs - 1) / (256 * kPairs);
      const size_t lds = (size_t)(Co * kChunk + Ci * (kChunk + 4)) * sizeof(double);
      hipLaunchKernelGGL(k_conv_bwd_weight_part, dim3(nbx, ngrp), dim3(256), lds, k->stream,
                         (const double *)g, Co, in, Ci, J, B, k->wpart);
      const int n = Co * Ci * KW;
      hipLaunchKernelGGL(k_conv_bwd_weight_sum, dim3((n + 63) / 64), dim3(64), 0, k->stream,
                         (const double *)k->wpart, n, nbx, k->gw + k->woff[l]);
    } else {
      hipLaunchKernelGGL(k_conv_bwd_weight, dim3(Co, Ci), dim3(256), 0, k->stream,
                         (const double *)g, Co, in, Ci, J, B, k->gw + k->woff[l]);
    }
    if (l > 0) {
      // (l > 0: Ci is the hidden width, a multiple of 8)
      hipLaunchKernelGGL(k_conv_bwd_data<8>, dim3((J + 255) / 256, Ci / 8, B), dim3(256), 0,
                         k->stream, (const double *)g, Co, J, (const double *)(k->w + k->woff[l]),
                         Ci, (const double *)k->act[l], gn);
      std::swap(g, gn);
    }
  }
  CK(k, hipGetLastError());
  return OCI_OK;
}

}  // namespace

extern "C" int oci_corrector_create(int32_t c_in, int32_t c_out, int32_t max_batch,
                                    int32_t max_cells, void *hip_stream, oci_corrector **out) {
  if (!out) return OCI_EINVAL;
  *out = nullptr;
  if (c_in < COT || c_out < COT || c_in % COT || c_out % COT || c_in > 1024 || c_out > 1024 ||
      max_batch < 1 || max_cells < 1 || (int64_t)max_batch * max_cells > ((int64_t)1 << 31))
    return OCI_EINVAL;
  oci_corrector *k = new oci_corrector();
  k->c_in = c_in;
  k->c_out = c_out;
  k->max_batch = max_batch;
  k->max_cells = max_cells;
  k->stream = (hipStream_t)hip_stream;
  k->chans[0] = c_in;
  for (int l = 1; l < NL; ++l) k->chans[l] = HID;
  k->chans[NL] = c_out;
  for (int l = 0; l < NL; ++l)
    k->woff[l + 1] = k->woff[l] + (size_t)k->chans[l + 1] * k->chans[l] * KW;
  const size_t nw = k->woff[NL];
  const size_t per = (size_t)max_batch * max_cells;
  const size_t gmax = per * (size_t)std::max(HID, std::max(c_out, c_in));
  bool ok = hipMalloc(&k->w, nw * sizeof(double)) == hipSuccess &&
            hipMalloc(&k->gw, nw * sizeof(double)) == hipSuccess &&
            hipMalloc(&k->m, nw * sizeof(double)) == hipSuccess &&
            hipMalloc(&k->v, nw * sizeof(double)) == hipSuccess &&
            hipMalloc(&k->y, per * c_out * sizeof(double)) == hipSuccess &&
            hipMalloc(&k->g0, gmax * sizeof(double)) == hipSuccess &&
            hipMalloc(&k->g1, gmax * sizeof(double)) == hipSuccess &&
            hipMalloc(&k->part, kPartBlocks * sizeof(double)) == hipSuccess &&
            hipMalloc(&k->loss, sizeof(double)) == hipSuccess &&
            hipMalloc(&k->wpart, (size_t)kTileCh * kTileCh * KW * kWgtBlocks * sizeof(double)) ==
                hipSuccess;
  for (int l = 1; ok && l < NL; ++l)
    ok = hipMalloc(&k->act[l], per * HID * sizeof(double)) == hipSuccess;
  ok = ok && hipMalloc(&k->w32, nw * sizeof(float)) == hipSuccess;
  for (int i = 0; ok && i < 2; ++i)
    ok = hipMalloc(&k->h32[i], per * HID * sizeof(float)) == hipSuccess;
  if (!ok) {
    oci_corrector_destroy(k);
    return OCI_ENOMEM;
  }
  // zero weights and moments until set_weights
  if (hipMemsetAsync(k->w, 0, nw * sizeof(double), k->stream) != hipSuccess ||
      hipMemsetAsync(k->m, 0, nw * sizeof(double), k->stream) != hipSuccess ||
      hipMemsetAsync(k->v, 0, nw * sizeof(double), k->stream) != hipSuccess ||
      hipStreamSynchronize(k->stream) != hipSuccess) {
    oci_corrector_destroy(k);
    return OCI_EDEVICE;
  }
  *out = k;
  return OCI_OK;
}

extern "C" int64_t oci_corrector_num_weights(const oci_corrector *k) {
  return k ? (int64_t)k->woff[NL] : (int64_t)OCI_EINVAL;
}

extern "C" int oci_corrector_set_weights(oci_corrector *k, const double *w) {
  if (!k || !w) return cfail(k, OCI_EINVAL, "NULL argument");
  const size_t nw = k->woff[NL];
  CK(k, hipMemcpyAsync(k->w, w, nw * sizeof(double), hipMemcpyHostToDevice, k->stream));
  CK(k, hipMemsetAsync(k->m, 0, nw * sizeof(double), k->stream));
  CK(k, hipMemsetAsync(k->v, 0, nw * sizeof(double), k->stream));
  CK(k, hipStreamSynchronize(k->stream));
  k->adam_t = 0;
  k->w32_stale = true;
  return OCI_OK;
}

extern "C" int oci_corrector_get_weights(oci_corrector *k, double *w) {
  if (!k || !w) return cfail(k, OCI_EINVAL, "NULL argument");
  CK(k, hipMemcpyAsync(w, k->w, k->woff[NL] * sizeof(double), hipMemcpyDeviceToHost, k->stream));
  CK(k, hipStreamSynchronize(k->stream));
  return OCI_OK;
}

extern "C" int oci_corrector_forward(oci_corrector *k, const double *x, int32_t batch,
                                     int32_t cells, double *y) {
  if (!k || !x || !y) return cfail(k, OCI_EINVAL, "NULL argument");
  int rc = check_shape(k, batch, cells);
  if (rc) return rc;
  return forward(k, x, batch, cells, y);
}

extern "C" int oci_corrector_grad(oci_corrector *k, const double *x, const double *target,
                                  int32_t batch, int32_t cells, double *loss, double *grad) {
  if (!k || !x || !target) return cfail(k, OCI_EINVAL, "NULL argument");
  int rc = check_shape(k, batch, cells);
  if (rc) return rc;
  rc = gradient(k, x, target, batch, cells);
  if (rc) return rc;
  if (loss) CK(k, hipMemcpyAsync(loss, k->loss, sizeof(double), hipMemcpyDeviceToHost, k->stream));
  if (grad)
    CK(k, hipMemcpyAsync(grad, k->gw, k->woff[NL] * sizeof(double), hipMemcpyDeviceToHost,
                         k->stream));
  CK(k, hipStreamSynchronize(k->stream));
  return OCI_OK;
}

extern "C" int oci_corrector_train_step(oci_corrector *k, const double *x, const double *target,
                                        int32_t batch, int32_t cells, double lr, double *loss) {
  if (!k || !x || !target) return cfail(k, OCI_EINVAL, "NULL argument");
  if (!(lr > 0.0) || !std::isfinite(lr)) return cfail(k, OCI_EINVAL, "learning rate must be > 0");
  int rc = check_shape(k, batch, cells);
  if (rc) return rc;
  rc = gradient(k, x, target, batch, cells);
  if (rc) return rc;
  const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
  k->adam_t += 1;
  const double bc1 = 1.0 - std::pow(b1, (double)k->adam_t);
  const double bc2 = 1.0 - std::pow(b2, (double)k->adam_t);
  hipLaunchKernelGGL(k_adam, dim3(64), dim3(256), 0, k->stream, k->w, (const double *)k->gw, k->m,
                     k->v, k->woff[NL], lr, b1, b2, eps, bc1, bc2);
  k->w32_stale = true;
  CK(k, hipGetLastError());
  if (loss) CK(k, hipMemcpyAsync(loss, k->loss, sizeof(double), hipMemcpyDeviceToHost, k->stream));
  CK(k, hipStreamSynchronize(k->stream));
  return OCI_OK;
}

extern "C" const char *oci_corrector_last_error(const oci_corrector *k) {
  return k ? k->err.c_str() : "corrector is NULL";
}

extern "C" void oci_corrector_destroy(oci_corrector *k) {
  if (!k) return;
  (void)hipStreamSynchronize(k->stream);
  double *bufs[] = {k->w, k->gw, k->m, k->v, k->y, k->g0, k->g1, k->part, k->loss,
                    k->wpart, k->act[1], k->act[2], k->act[3]};
  for (double *p : bufs)
    if (p) (void)hipFree(p);
  float *fbufs[] = {k->w32, k->h32[0], k->h32[1]};
  for (float *p : fbufs)
    if (p) (void)hipFree(p);
  delete k;
}

// ---------------------------------------------------------------------------
// FP32 inference on the matrix cores
// ---------------------------------------------------------------------------
namespace {

// y = f(x) in FP32 for x [B][c_in][J] on stream st (the FP32 weights
// refreshed first when stale, on the same stream).
int infer32(oci_corrector *k, hipStream_t st, const float *x, int B, int J, float *y) {
  if (k->w32_stale) {
    hipLaunchKernelGGL(k_to_f32, dim3(64), dim3(256), 0, st, (const double *)k->w, k->woff[NL],
                       k->w32);
    k->w32_stale = false;
  }
  const float *in = x;
  for (int l = 0; l < NL; ++l) {
    const int Ci = k->chans[l], Co = k->chans[l + 1];
    float *o = l == NL - 1 ? y : k->h32[l & 1];
    const int MT = (Co + 15) / 16, KP = (Ci * KW + 3) & ~3;
    const size_t lds = (size_t)(MT * 16 * KP + Ci * (kC32 + KW - 1)) * sizeof(float);
    hipLaunchKernelGGL(k_conv_fwd32, dim3((J + kC32 - 1) / kC32, 1, B), dim3(256), lds, st, in, Ci,
                       J, (const float *)(k->w32 + k->woff[l]), Co, o, l < NL - 1 ? 1 : 0);
    in = o;
  }
  CK(k, hipGetLastError());
  return OCI_OK;
}

}  // namespace

int occ_infer32(oci_corrector *k, hipStream_t st, const float *x, int cells, float *y) {
  if (!k || !x || !y) return OCI_EINVAL;
  if (cells < 1 || (int64_t)cells > (int64_t)k->max_batch * k->max_cells) return OCI_EINVAL;
  return infer32(k, st, x, 1, cells, y);
}

int occ_channels(const oci_corrector *k, int *c_in, int *c_out, int64_t *max_cells) {
  if (!k) return OCI_EINVAL;
  *c_in = k->c_in;
  *c_out = k->c_out;
  *max_cells = (int64_t)k->max_batch * k->max_cells;
  return OCI_OK;
}

extern "C" int oci_corrector_forward32(oci_corrector *k, const float *x, int32_t batch,
                                       int32_t cells, float *y) {
  if (!k || !x || !y) return cfail(k, OCI_EINVAL, "NULL argument");
  if (k->c_in > 32 || k->c_out > 32)
    return cfail(k, OCI_EINVAL, "FP32 inference takes at most 32 input and output channels");
  int rc = check_shape(k, batch, cells);
  if (rc) return rc;
  return infer32(k, k->stream, x, batch, cells, y);
}

// ---------------------------------------------------------------------------
// Allocation-free inference
// ---------------------------------------------------------------------------
// The hidden activations of oci_corrector_forward_noalloc live in one
// file-scope device array (each GPU the library runs on holds its own copy
// until the process ends): two [batch][32][cells] buffers used in turn, so a
// call handles batch * cells <= kNoAllocCells.  Host code never passes the
// array's name to a kernel (in host code it is a stand-in, not a device
// address): its device address is looked up once per device with
// hipGetSymbolAddress, with that device current, and kept.
namespace occ {
constexpr int64_t kNoAllocCells = 65536;
constexpr size_t kScratchDoubles = (size_t)2 * HID * kNoAllocCells;   // 32 MiB
constexpr int kMaxDevices = 64;
}  // namespace occ

static __device__ __align__(256) double scratch[occ::kScratchDoubles];

namespace {

std::mutex g_scratch_mu;
double *g_scratch_ptr[occ::kMaxDevices] = {};

// Device address of this device's scratch array (looked up on first use).
hipError_t scratch_of_current_device(double **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= occ::kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = static_cast<double *>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" int oci_corrector_forward_noalloc(const double *w, int32_t c_in, int32_t c_out,
                                             const double *x, int32_t batch, int32_t cells,
                                             double *y, void *hip_stream) {
  if (!w || !x || !y) return OCI_EINVAL;
  if (c_in < COT || c_out < COT || c_in % COT || c_out % COT || c_in > 1024 || c_out > 1024)
    return OCI_EINVAL;
  if (batch < 1 || cells < 1 || (int64_t)batch * cells > kNoAllocCells) return OCI_EINVAL;
  double *scr = nullptr;
  if (scratch_of_current_device(&scr) != hipSuccess) return OCI_EDEVICE;
  int chans[NL + 1];
  size_t woff[NL + 1] = {};
  chans[0] = c_in;
  for (int l = 1; l < NL; ++l) chans[l] = HID;
  chans[NL] = c_out;
  for (int l = 0; l < NL; ++l) woff[l + 1] = woff[l] + (size_t)chans[l + 1] * chans[l] * KW;
  // layer outputs: scr, scr + per, scr (layer 2 reads the second buffer)
  const size_t per = (size_t)HID * batch * cells;
  double *act[NL] = {nullptr, scr, scr + per, scr};
  const hipError_t e = launch_forward(static_cast<hipStream_t>(hip_stream), w, woff, chans, x,
                                      batch, cells, y, act);
  return e == hipSuccess ? OCI_OK : OCI_EDEVICE;
}
