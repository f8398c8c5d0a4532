// Gaussian-hill bias on the device, FP64: evaluation of V and dV/ds, and the
// deposition of one well-tempered hill.  Fixed-order sums (thread -> wave ->
// block -> last block over the block partials), so results are reproducible.
#include "gm_device.h"

namespace gm {

// --------------------------------------------------------------------------
// Gaussian-hill bias (FP64): evaluation, or deposition of one hill.
// --------------------------------------------------------------------------
// s - c, or its nearest periodic image for a periodic dimension.
__device__ __forceinline__ double cv_delta(double s, double c, double period) {
  const double x = s - c;
  return period > 0.0 ? x - period * rint(x / period) : x;
}

__device__ __forceinline__ void bias_body(const BiasArgs& a, int32_t blk, int32_t nblk) {
  __shared__ double red[kBlock / 64];
  const int64_t K = *a.count;
  double s[2] = {a.s[0], a.dims > 1 ? a.s[1] : 0.0};
  double v = 0.0, g0 = 0.0, g1 = 0.0;
  const int64_t stride = (int64_t)nblk * blockDim.x;
  for (int64_t k = (int64_t)blk * blockDim.x + threadIdx.x; k < K; k += stride) {
    const double x0 = cv_delta(s[0], a.centres[k * a.dims], a.period[0]);
    double arg = x0 * x0 * a.inv2s2[0];
    double x1 = 0.0;
    if (a.dims > 1) {
      x1 = cv_delta(s[1], a.centres[k * a.dims + 1], a.period[1]);
      arg += x1 * x1 * a.inv2s2[1];
    }
    const double e = a.heights[k] * exp(-arg);
    v += e;
    g0 -= e * x0 * a.invs2[0];
    g1 -= e * x1 * a.invs2[1];
  }
  v = block_sum(v, red);
  g0 = block_sum(g0, red);
  if (a.dims > 1) g1 = block_sum(g1, red);
  if (threadIdx.x == 0) {
    a.part[blk * 3 + 0] = v;
    a.part[blk * 3 + 1] = g0;
    a.part[blk * 3 + 2] = g1;
  }
}

// Fixed-order sum of the bias partials (its own launch); V and dV/ds, or the
// deposit of one hill.
__device__ __forceinline__ void bias_finish_body(const BiasArgs& a, int32_t nblk) {
  __shared__ double red[kBlock / 64];
  const int64_t K = *a.count;
  double V = 0.0, G0 = 0.0, G1 = 0.0;
  for (int64_t i = threadIdx.x; i < (int64_t)nblk; i += blockDim.x) {
    V += a.part[i * 3 + 0];
    G0 += a.part[i * 3 + 1];
    G1 += a.part[i * 3 + 2];
  }
  V = block_sum(V, red);
  G0 = block_sum(G0, red);
  if (a.dims > 1) G1 = block_sum(G1, red);
  if (threadIdx.x == 0) {
    if (!isfinite(V)) atomicOr(a.err, kErrNonFinite);
    if (a.deposit) {
      const double h = a.wt_scale == 0.0 ? a.w0 : a.w0 * exp(-V * a.wt_scale);
      if (K < a.capacity) {
        for (int d = 0; d < a.dims; d++) a.centres[K * a.dims + d] = a.s[d];
        a.heights[K] = h;
        *a.count = K + 1;
      } else {
        atomicOr(a.err, kErrCapacity);
      }
    } else {
      if (a.V_out) a.V_out[0] = V;
      if (a.dV_out) {
        a.dV_out[0] = G0;
        if (a.dims > 1) a.dV_out[1] = G1;
      }
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_bias(BiasArgs a) { bias_body(a, blockIdx.x, gridDim.x); }

__global__ __launch_bounds__(kBlock) void k_bias_finish(BiasArgs a, int32_t nblk) { bias_finish_body(a, nblk); }

__global__ __launch_bounds__(kBlock) void k_bias_finish_batch(const BiasArgs* __restrict__ tab,
                                                              const int32_t* __restrict__ blk_start) {
  const int32_t w = blockIdx.x;
  bias_finish_body(tab[w], blk_start[w + 1] - blk_start[w]);
}

// One launch for many walkers: workgroup g serves walker w with
// blk_start[w] <= g < blk_start[w+1].
__global__ __launch_bounds__(kBlock) void k_bias_batch(const BiasArgs* __restrict__ tab,
                                                       const int32_t* __restrict__ blk_start, int32_t W) {
  const int64_t g = blockIdx.x;
  int32_t lo = 0, hi = W;
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (blk_start[mid] <= g) lo = mid; else hi = mid;
  }
  bias_body(tab[lo], (int32_t)(g - blk_start[lo]), blk_start[lo + 1] - blk_start[lo]);
}

hipError_t launch_bias_batch(const BiasArgs* tab, const int32_t* blk_start, int32_t W, int32_t blocks,
                             hipStream_t st) {
  k_bias_batch<<<(unsigned)blocks, kBlock, 0, st>>>(tab, blk_start, W);
  k_bias_finish_batch<<<(unsigned)W, kBlock, 0, st>>>(tab, blk_start);
  return hipGetLastError();
}

// The same for a subset of a batch's walkers named by value.
__global__ __launch_bounds__(kBlock) void k_bias_subset(BiasSubset s) {
  const int32_t g = blockIdx.x;
  int32_t lo = 0, hi = s.k;
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (s.blk[mid] <= g) lo = mid; else hi = mid;
  }
  bias_body(*s.tab[lo], g - s.blk[lo], s.blk[lo + 1] - s.blk[lo]);
}

__global__ __launch_bounds__(kBlock) void k_bias_finish_subset(BiasSubset s) {
  const int32_t w = blockIdx.x;
  bias_finish_body(*s.tab[w], s.blk[w + 1] - s.blk[w]);
}

hipError_t launch_bias_subset(const BiasSubset& s, hipStream_t st) {
  if (s.k < 1) return hipSuccess;
  k_bias_subset<<<(unsigned)s.blk[s.k], kBlock, 0, st>>>(s);
  k_bias_finish_subset<<<(unsigned)s.k, kBlock, 0, st>>>(s);
  return hipGetLastError();
}

// CV, bias and dV/ds of every walker of a batch into dense arrays (second
// columns hold the contexts' zero second entries for 1-D CVs).
__global__ __launch_bounds__(kBlock) void k_batch_values(const double* const* __restrict__ tab, int32_t W, double* s,
                                                         double* V, double* dV) {
  const int32_t w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  const double* sw = tab[3 * w];
  const double* vw = tab[3 * w + 1];
  const double* dw = tab[3 * w + 2];
  if (s) {
    s[2 * w] = sw[0];
    s[2 * w + 1] = sw[1];
  }
  if (V) V[w] = vw[0];
  if (dV) {
    dV[2 * w] = dw[0];
    dV[2 * w + 1] = dw[1];
  }
}

hipError_t launch_batch_values(const double* const* tab, int32_t W, double* s, double* V, double* dV, hipStream_t st) {
  k_batch_values<<<(unsigned)((W + kBlock - 1) / kBlock), kBlock, 0, st>>>(tab, W, s, V, dV);
  return hipGetLastError();
}

hipError_t launch_bias(const BiasArgs& a, int blocks, hipStream_t st) {
  k_bias<<<(unsigned)blocks, kBlock, 0, st>>>(a);
  k_bias_finish<<<1, kBlock, 0, st>>>(a, blocks);
  return hipGetLastError();
}

}  // namespace gm
