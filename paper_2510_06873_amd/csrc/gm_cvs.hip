// Collective variables of a few atoms and free-energy surfaces.
//
//  * torsion angles of atom quadruples (paper, Results, "Alanine dipeptide
//    torsion": the backbone Phi and Psi), IUPAC sign, and their bias forces;
//  * the distance from one atom to the nearest atom of a set (paper, Results,
//    "Water dissociation on rutile (110) surface": a surface oxygen and its
//    nearest hydrogen), and its bias forces;
//  * the free energy of a biased trajectory by reweighting (paper, Methods:
//    P(s) from the biased averages of delta(s - s(R)) e^{beta V} and
//    e^{beta V}, F = -(1/beta) log P), and from the deposited hills on a grid.
//
// These are latency-bound, so each is a small launch in FP64 on the FP32
// coordinates.  Atom indices are device arrays; an index outside [0, n)
// gives NaN for the CV it belongs to and no force (it is never dereferenced).
#include <mutex>

#include "gm_device.h"

namespace gm {
namespace {

constexpr int kSmallBlock = 256;
constexpr int kNearBlock = 1024;
constexpr int kFesLdsBins = 16384;  // per-block histograms in LDS up to this many bins

struct Box64 {
  double L[3];
};

// Minimum image of x_j - x_i in FP64 (no contraction): d -= L rint(d / L).
__device__ __forceinline__ void pair64(const float4* pos, int32_t i, int32_t j, const Box64& b, double d[3]) {
#pragma clang fp contract(off)
  const float4 pi = pos[i], pj = pos[j];
  const double v[3] = {(double)pj.x - (double)pi.x, (double)pj.y - (double)pi.y, (double)pj.z - (double)pi.z};
#pragma unroll
  for (int a = 0; a < 3; a++) d[a] = v[a] - b.L[a] * rint(v[a] / b.L[a]);
}

// r^2 = (dx dx + dy dy) + dz dz, each product rounded (no contraction).
__device__ __forceinline__ double dist2_nofma(const double d[3]) {
#pragma clang fp contract(off)
  return d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
}

__device__ __forceinline__ void cross(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

__device__ __forceinline__ double dot(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Torsion of atoms q[0..3]: phi = atan2(|b2| b1.n2, n1.n2), b1 = x2 - x1,
// b2 = x3 - x2, b3 = x4 - x3, n1 = b1 x b2, n2 = b2 x b3.  With grad != NULL
// also dphi/dx of the four atoms: the ends move along the plane normals,
//   g1 = -|b2|/|n1|^2 n1,  g4 = |b2|/|n2|^2 n2,
// and with p = b1.b2/|b2|^2, q = b3.b2/|b2|^2 the middle atoms take
//   g2 = -(1 + p) g1 + q g4,  g3 = -(1 + q) g4 + p g1.
__device__ double torsion(const float4* pos, const int32_t q[4], const Box64& box, double grad[4][3]) {
  double b1[3], b2[3], b3[3], n1[3], n2[3];
  pair64(pos, q[0], q[1], box, b1);
  pair64(pos, q[1], q[2], box, b2);
  pair64(pos, q[2], q[3], box, b3);
  cross(b1, b2, n1);
  cross(b2, b3, n2);
  const double lb2 = sqrt(dot(b2, b2));
  if (grad) {
    const double b2b2 = lb2 * lb2, p = dot(b1, b2) / b2b2, qq = dot(b3, b2) / b2b2;
    const double c1 = -lb2 / dot(n1, n1), c4 = lb2 / dot(n2, n2);
#pragma unroll
    for (int a = 0; a < 3; a++) {
      const double g1 = c1 * n1[a], g4 = c4 * n2[a];
      grad[0][a] = g1;
      grad[1][a] = -(1.0 + p) * g1 + qq * g4;
      grad[2][a] = -(1.0 + qq) * g4 + p * g1;
      grad[3][a] = g4;
    }
  }
  return atan2(lb2 * dot(b1, n2), dot(n1, n2));
}

__device__ __forceinline__ bool load_quad(const int32_t* quads, int32_t t, int64_t n, int32_t q[4]) {
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    q[k] = quads[4 * t + k];
    ok = ok && q[k] >= 0 && q[k] < n;
  }
  return ok;
}

__global__ __launch_bounds__(kSmallBlock) void k_torsions(const float4* __restrict__ pos, int64_t n,
                                                          const int32_t* __restrict__ quads, int32_t count,
                                                          Box64 box, double* __restrict__ phi) {
  const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  int32_t q[4];
  phi[t] = load_quad(quads, t, n, q) ? torsion(pos, q, box, nullptr) : __builtin_nan("");
}

// F_i -= sum_t dV/dphi_t dphi_t/dx_i, one thread in torsion order (torsions
// share atoms; the order fixes the result).
template <typename F>
__global__ void k_torsion_forces(const float4* __restrict__ pos, int64_t n, const int32_t* __restrict__ quads,
                                 int32_t count, Box64 box, const double* __restrict__ dV, F* force) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  for (int32_t t = 0; t < count; t++) {
    int32_t q[4];
    if (!load_quad(quads, t, n, q)) continue;
    double g[4][3];
    torsion(pos, q, box, g);
    const double f = dV[t];
    for (int k = 0; k < 4; k++) {
      F* r = force + 4 * (int64_t)q[k];
      r[0] = (F)((double)r[0] - f * g[k][0]);
      r[1] = (F)((double)r[1] - f * g[k][1]);
      r[2] = (F)((double)r[2] - f * g[k][2]);
    }
  }
}

// Nearest member of the set to the centre: (r, set position) minimised
// lexicographically, i.e. the earliest member among equal distances; the
// centre itself is skipped.  mode 0 writes s and the atom; mode 1 adds the
// bias force: F_centre += dV/ds u, F_nearest -= dV/ds u (u from the centre to
// the nearest atom).
template <typename F>
__global__ __launch_bounds__(kNearBlock) void k_nearest(const float4* __restrict__ pos, int64_t n, int32_t centre,
                                                        const int32_t* __restrict__ members, int32_t count, Box64 box,
                                                        double* s_out, int32_t* atom_out, const double* dV, F* force) {
  __shared__ double rs[kNearBlock];
  __shared__ int32_t ks[kNearBlock];
  __shared__ int32_t bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  double best = __builtin_inf();
  int32_t bk = INT32_MAX;
  for (int32_t k = threadIdx.x; k < count; k += blockDim.x) {
    const int32_t j = members[k];
    if (j < 0 || j >= n) {
      bad = 1;
      continue;
    }
    if (j == centre) continue;
    double d[3];
    pair64(pos, centre, j, box, d);
    const double r = sqrt(dist2_nofma(d));
    if (r < best) {  // k increases within a thread: the first minimum stays
      best = r;
      bk = k;
    }
  }
  rs[threadIdx.x] = best;
  ks[threadIdx.x] = bk;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      const double r2 = rs[threadIdx.x + h];
      const int32_t k2 = ks[threadIdx.x + h];
      if (r2 < rs[threadIdx.x] || (r2 == rs[threadIdx.x] && k2 < ks[threadIdx.x])) {
        rs[threadIdx.x] = r2;
        ks[threadIdx.x] = k2;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const bool ok = !bad && ks[0] != INT32_MAX;
  const int32_t j = ok ? members[ks[0]] : -1;
  if (s_out) {
    s_out[0] = ok ? rs[0] : __builtin_nan("");
    if (atom_out) atom_out[0] = j;
  }
  if (force && ok) {
    double d[3];
    pair64(pos, centre, j, box, d);
    const double f = dV[0] / rs[0];
    F* rc = force + 4 * (int64_t)centre;
    F* rn = force + 4 * (int64_t)j;
    for (int a = 0; a < 3; a++) {
      rc[a] = (F)((double)rc[a] + f * d[a]);
      rn[a] = (F)((double)rn[a] - f * d[a]);
    }
  }
}

// --------------------------------------------------------------------------
// Free energy by reweighting.  V_max by a max reduction (order-free), the
// denominator sum_t w_t by fixed-order block partials, the per-bin numerators
// by per-block LDS histograms merged with FP64 atomics (reproducible to about
// 1e-15 relative, not bit for bit), then F = -kBT log(num / den).
// --------------------------------------------------------------------------
struct FesArgs {
  const double* s;  // [T][dims]
  const double* V;  // [T]
  int64_t T;
  int32_t dims;
  double lo[2], width[2];
  int32_t nb[2];
  int32_t nbins;
  double kBT;
  double* vmax_part;  // [blocks]
  double* den_part;   // [blocks]
  double* num;        // [nbins]
  double* F;          // [nbins]
};

__device__ __forceinline__ int32_t fes_bin(const FesArgs& a, int64_t t) {
  int32_t bin = 0, stride = 1;
  for (int d = 0; d < a.dims; d++) {
    const double x = floor((a.s[t * a.dims + d] - a.lo[d]) / a.width[d]);
    if (!(x >= 0.0 && x < (double)a.nb[d])) return -1;
    bin += (int32_t)x * stride;
    stride *= a.nb[d];
  }
  return bin;
}

__global__ __launch_bounds__(kSmallBlock) void k_fes_vmax(FesArgs a) {
  __shared__ double red[kSmallBlock];
  double m = -__builtin_inf();
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < a.T; t += (int64_t)gridDim.x * blockDim.x)
    m = fmax(m, a.V[t]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) a.vmax_part[blockIdx.x] = red[0];
}

template <bool LDS_HIST>
__global__ __launch_bounds__(kSmallBlock) void k_fes_accum(FesArgs a, int32_t nblk) {
  extern __shared__ double hist[];
  __shared__ double red[kSmallBlock / 64];
  double vmax = -__builtin_inf();
  for (int32_t i = 0; i < nblk; i++) vmax = fmax(vmax, a.vmax_part[i]);
  if (LDS_HIST) {
    for (int32_t b = threadIdx.x; b < a.nbins; b += blockDim.x) hist[b] = 0.0;
    __syncthreads();
  }
  double den = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < a.T; t += (int64_t)gridDim.x * blockDim.x) {
    const double w = exp((a.V[t] - vmax) / a.kBT);
    den += w;
    const int32_t bin = fes_bin(a, t);
    if (bin >= 0) atomicAdd(LDS_HIST ? &hist[bin] : &a.num[bin], w);
  }
  den = block_sum(den, red);
  if (threadIdx.x == 0) a.den_part[blockIdx.x] = den;
  if (LDS_HIST) {
    __syncthreads();
    for (int32_t b = threadIdx.x; b < a.nbins; b += blockDim.x)
      if (hist[b] != 0.0) atomicAdd(&a.num[b], hist[b]);
  }
}

__global__ __launch_bounds__(kSmallBlock) void k_fes_out(FesArgs a, int32_t nblk) {
  double den = 0.0;  // the same fixed order in every thread
  for (int32_t i = 0; i < nblk; i++) den += a.den_part[i];
  for (int32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < a.nbins; b += gridDim.x * blockDim.x) {
    const double p = a.num[b] / den;
    a.F[b] = a.num[b] > 0.0 ? -a.kBT * log(p) : __builtin_inf();
  }
}

__global__ __launch_bounds__(kSmallBlock) void k_zero_f64(double* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// F = -scale V on the grid of bin centres, hills in index order.  Every
// grid point of a workgroup reads every hill, so the hills pass through LDS
// in tiles (one coalesced read of each hill per workgroup instead of one per
// wave).
constexpr int kHillTile = 512;

__global__ __launch_bounds__(kSmallBlock) void k_fes_hills(BiasArgs b, double lo0, double lo1, double w0,
                                                           double w1, int32_t nb0, int32_t nbins, double scale,
                                                           double* F) {
  __shared__ double tc0[kHillTile], tc1[kHillTile], th[kHillTile];
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t ic = i < nbins ? i : nbins - 1;  // threads past the grid help stage, store nothing
  const double g0 = lo0 + ((ic % nb0) + 0.5) * w0, g1 = lo1 + ((ic / nb0) + 0.5) * w1;
  const int64_t K = *b.count;
  const bool two = b.dims > 1;
  double v = 0.0;
  for (int64_t t0 = 0; t0 < K; t0 += kHillTile) {
    const int32_t n = (int32_t)(K - t0 < kHillTile ? K - t0 : kHillTile);
    __syncthreads();  // the previous tile is no longer read
    for (int32_t q = threadIdx.x; q < n; q += blockDim.x) {
      tc0[q] = b.centres[(t0 + q) * b.dims];
      tc1[q] = two ? b.centres[(t0 + q) * b.dims + 1] : 0.0;
      th[q] = b.heights[t0 + q];
    }
    __syncthreads();
    for (int32_t q = 0; q < n; q++) {
      double x = g0 - tc0[q];
      if (b.period[0] > 0.0) x -= b.period[0] * rint(x / b.period[0]);
      double arg = x * x * b.inv2s2[0];
      if (two) {
        double y = g1 - tc1[q];
        if (b.period[1] > 0.0) y -= b.period[1] * rint(y / b.period[1]);
        arg += y * y * b.inv2s2[1];
      }
      v += th[q] * exp(-arg);
    }
  }
  if (i < nbins) F[i] = -scale * v;
}

unsigned grid_for(int64_t n, int block, int64_t cap) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

}  // namespace

hipError_t launch_torsions(const float4* pos, int64_t n, const int32_t* quads, int32_t count, const double* box,
                           double* phi, hipStream_t st) {
  const Box64 b{{box[0], box[1], box[2]}};
  if (count > 0) k_torsions<<<grid_for(count, kSmallBlock, 1 << 20), kSmallBlock, 0, st>>>(pos, n, quads, count, b, phi);
  return hipGetLastError();
}

hipError_t launch_torsion_forces(const float4* pos, int64_t n, const int32_t* quads, int32_t count, const double* box,
                                 const double* dV, void* force, bool fp64, hipStream_t st) {
  const Box64 b{{box[0], box[1], box[2]}};
  if (count > 0) {
    if (fp64)
      k_torsion_forces<double><<<1, 64, 0, st>>>(pos, n, quads, count, b, dV, reinterpret_cast<double*>(force));
    else
      k_torsion_forces<float><<<1, 64, 0, st>>>(pos, n, quads, count, b, dV, reinterpret_cast<float*>(force));
  }
  return hipGetLastError();
}

hipError_t launch_nearest(const float4* pos, int64_t n, int32_t centre, const int32_t* members, int32_t count,
                          const double* box, double* s, int32_t* atom, const double* dV, void* force, bool fp64,
                          hipStream_t st) {
  const Box64 b{{box[0], box[1], box[2]}};
  if (fp64)
    k_nearest<double><<<1, kNearBlock, 0, st>>>(pos, n, centre, members, count, b, s, atom, dV,
                                                 reinterpret_cast<double*>(force));
  else
    k_nearest<float><<<1, kNearBlock, 0, st>>>(pos, n, centre, members, count, b, s, atom, dV,
                                                reinterpret_cast<float*>(force));
  return hipGetLastError();
}

// Scratch of the allocation-free reweighting: one array per device for the
// life of the process, shared by every call on that device (calls that
// overlap on one device race on it).  Host code uses only the device address
// hipGetSymbolAddress returns for it, looked up once per device.
constexpr size_t kFesScratchDoubles = 2 * 1024 + (size_t)kFesNoAllocMaxBins;
static __device__ __align__(256) double scratch[kFesScratchDoubles];

namespace {

FesArgs fes_args(const double* s, const double* V, int64_t T, int32_t dims, const double* lo, const double* hi,
                 const int32_t* nb, double kBT, double* F) {
  FesArgs a{};
  a.s = s;
  a.V = V;
  a.T = T;
  a.dims = dims;
  a.nbins = 1;
  for (int d = 0; d < dims; d++) {
    a.lo[d] = lo[d];
    a.width[d] = (hi[d] - lo[d]) / nb[d];
    a.nb[d] = nb[d];
    a.nbins *= nb[d];
  }
  a.kBT = kBT;
  a.F = F;
  return a;
}

// Workgroups of the sample passes and the doubles of scratch they need: the
// per-workgroup maxima and denominators, then the per-bin numerators.
unsigned fes_blocks(int64_t T) { return grid_for(T, kSmallBlock, 1024); }
size_t fes_scratch_doubles(int64_t T, int32_t nbins) { return 2 * (size_t)fes_blocks(T) + (size_t)nbins; }

// The reweighting kernels over a scratch of fes_scratch_doubles(T, nbins)
// doubles; every value of it that they read is written first (the
// numerators by k_zero_f64, the partials by one workgroup each).
hipError_t enqueue_fes_reweight(FesArgs a, double* scratch, hipStream_t st) {
  const unsigned blocks = fes_blocks(a.T);
  a.vmax_part = scratch;
  a.den_part = a.vmax_part + blocks;
  a.num = a.den_part + blocks;
  k_zero_f64<<<grid_for(a.nbins, kSmallBlock, 4096), kSmallBlock, 0, st>>>(a.num, a.nbins);
  k_fes_vmax<<<blocks, kSmallBlock, 0, st>>>(a);
  if (a.nbins <= kFesLdsBins)
    k_fes_accum<true><<<blocks, kSmallBlock, (size_t)a.nbins * sizeof(double), st>>>(a, (int32_t)blocks);
  else
    k_fes_accum<false><<<blocks, kSmallBlock, 0, st>>>(a, (int32_t)blocks);
  k_fes_out<<<grid_for(a.nbins, kSmallBlock, 4096), kSmallBlock, 0, st>>>(a, (int32_t)blocks);
  return hipGetLastError();
}

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxScratchDevices] = {};

hipError_t scratch_on_current_device(double** out) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = reinterpret_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

hipError_t launch_fes_reweight(const double* s, const double* V, int64_t T, int32_t dims, const double* lo,
                               const double* hi, const int32_t* nb, double kBT, double* F, hipStream_t st) {
  const FesArgs a = fes_args(s, V, T, dims, lo, hi, nb, kBT, F);
  void* buf = nullptr;
  hipError_t e = hipMallocAsync(&buf, fes_scratch_doubles(T, a.nbins) * sizeof(double), st);
  if (e != hipSuccess) return e;
  e = enqueue_fes_reweight(a, reinterpret_cast<double*>(buf), st);
  const hipError_t f = hipFreeAsync(buf, st);
  return e != hipSuccess ? e : f;
}

hipError_t launch_fes_reweight_noalloc(const double* s, const double* V, int64_t T, int32_t dims, const double* lo,
                                       const double* hi, const int32_t* nb, double kBT, double* F, hipStream_t st) {
  const FesArgs a = fes_args(s, V, T, dims, lo, hi, nb, kBT, F);
  if (a.nbins > kFesNoAllocMaxBins || fes_scratch_doubles(T, a.nbins) > kFesScratchDoubles)
    return hipErrorInvalidValue;  // the caller checks the grid size first
  double* buf = nullptr;
  const hipError_t e = scratch_on_current_device(&buf);
  if (e != hipSuccess) return e;
  return enqueue_fes_reweight(a, buf, st);
}

hipError_t launch_fes_hills(const BiasArgs& b, const double* lo, const double* hi, const int32_t* nb, double scale,
                            double* F, hipStream_t st) {
  const int32_t nb0 = nb[0], nb1 = b.dims > 1 ? nb[1] : 1, nbins = nb0 * nb1;
  const double w0 = (hi[0] - lo[0]) / nb0, w1 = b.dims > 1 ? (hi[1] - lo[1]) / nb1 : 0.0;
  k_fes_hills<<<grid_for(nbins, kSmallBlock, 1 << 20), kSmallBlock, 0, st>>>(b, lo[0], b.dims > 1 ? lo[1] : 0.0, w0, w1,
                                                                             nb0, nbins, scale, F);
  return hipGetLastError();
}

void allow_fes_lds() {
  (void)hipFuncSetAttribute((const void*)k_fes_accum<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            kFesLdsBins * (int)sizeof(double));
  (void)hipGetLastError();
}

}  // namespace gm
