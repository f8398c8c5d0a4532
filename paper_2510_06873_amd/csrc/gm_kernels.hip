// HIP kernels of the metadynamics bias pipeline for gfx950.
//
// Layout: after each neighbour build the atoms are handled in cell-sorted
// order (position t holds the atom perm[t]); positions are gathered into that
// order once per step, so the neighbour gathers of one block touch a compact
// region of space.  Per-atom CV intermediates are 16-wide rows (64 B in FP32):
// one neighbour's q-hat row or adjoint row is one cache line.  Blocks are
// remapped so that each XCD (own L2) walks a contiguous range of sorted atoms.
//
// Reductions that define a result (the CV sums, the hill sums) are FP64 in a
// fixed order: per-thread value -> wavefront shuffle tree -> block -> the last
// block to finish sums the block partials by index.  No FP64 atomics, so the
// results are bitwise reproducible run to run.
#include <math.h>

#include "gm_internal.h"

namespace gm {

// --------------------------------------------------------------------------
// Small device helpers
// --------------------------------------------------------------------------
__device__ __forceinline__ float g_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double g_rsqrt(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float g_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double g_rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float g_exp(float x) { return __expf(x); }
__device__ __forceinline__ double g_exp(double x) { return exp(x); }
__device__ __forceinline__ float g_rint(float x) { return rintf(x); }
__device__ __forceinline__ double g_rint(double x) { return rint(x); }
__device__ __forceinline__ void g_sincos(float x, float* s, float* c) { sincosf(x, s, c); }
__device__ __forceinline__ void g_sincos(double x, double* s, double* c) { sincos(x, s, c); }
__device__ __forceinline__ float g_sqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double g_sqrt(double x) { return sqrt(x); }

template <typename T>
__device__ __forceinline__ T logistic(T x) {
  return g_rcp(T(1) + g_exp(-x));
}

// Logical block index: XCD x (= blockIdx % 8) gets the contiguous block range
// [x*G/8, (x+1)*G/8) so that neighbouring atoms share an L2.
__device__ __forceinline__ int64_t logical_block() {
  int64_t b = blockIdx.x;
  int64_t per = gridDim.x / kXcd;
  return (b % kXcd) * per + b / kXcd;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// Fixed-order block sum; the result is valid in thread 0.  All threads call.
__device__ __forceinline__ double block_sum(double v, double* lds) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) lds[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); i++) r += lds[i];
  __syncthreads();
  return r;
}

__device__ __forceinline__ void store_agent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double load_agent(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// True in every thread of the block that finishes last (all threads call).
__device__ __forceinline__ bool last_block_done(unsigned* ticket) {
  __shared__ int is_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned prev = atomicAdd(ticket, 1u);
    is_last = (prev == gridDim.x - 1) ? 1 : 0;
  }
  __syncthreads();
  if (is_last) __threadfence();
  return is_last != 0;
}

__device__ __forceinline__ void release_ticket(unsigned* ticket) {
  if (threadIdx.x == 0) atomicExch(ticket, 0u);
}

// Minimum image in T: d - L*rint(d/L), with L split in high and low parts so
// that an FP32 box length does not bias wrapped pairs.
template <typename T>
__device__ __forceinline__ T mic(T d, T L, T invL, T Llo) {
  T k = g_rint(d * invL);
  return (d - k * L) - k * Llo;
}

template <typename T>
__device__ __forceinline__ T pair_vec(const vec4_t<T>& pi, const vec4_t<T>& pj, const CvArgs<T>& a,
                                      T& dx, T& dy, T& dz) {
  dx = mic(pj.x - pi.x, a.L[0], a.invL[0], a.Llo[0]);
  dy = mic(pj.y - pi.y, a.L[1], a.invL[1], a.Llo[1]);
  dz = mic(pj.z - pi.z, a.L[2], a.invL[2], a.Llo[2]);
  return dx * dx + dy * dy + dz * dz;
}

// Cosine-tapered q6 weight f(r) and f'(r).
template <typename T>
__device__ __forceinline__ T taper_w(T r, const CvArgs<T>& a, T& df) {
  if (r <= a.taper_lo) {
    df = T(0);
    return T(1);
  }
  T s, c;
  g_sincos((r - a.taper_lo) * a.pi_over_D, &s, &c);
  df = -a.half_pi_over_D * s;
  return T(0.5) + T(0.5) * c;
}

template <typename T>
__device__ __forceinline__ void eval_E(const YCoef<T>& c, T z, T E[7]) {
  const T z2 = z * z;
  E[0] = c.e0[0] + z2 * (c.e0[1] + z2 * (c.e0[2] + z2 * c.e0[3]));
  E[1] = z * (c.e1[0] + z2 * (c.e1[1] + z2 * c.e1[2]));
  E[2] = c.e2[0] + z2 * (c.e2[1] + z2 * c.e2[2]);
  E[3] = z * (c.e3[0] + z2 * c.e3[1]);
  E[4] = c.e4[0] + z2 * c.e4[1];
  E[5] = z * c.e5;
  E[6] = c.e6;
}

// Q += f * v(u), v the real 13-vector of l = 6 harmonics:
// v_0 = E_0, v_{2m-1} = E_m Re (ux + i uy)^m, v_{2m} = E_m Im (ux + i uy)^m.
template <typename T>
__device__ __forceinline__ void accumulate_y(const YCoef<T>& c, T ux, T uy, T uz, T f, T Q[13]) {
  T E[7];
  eval_E(c, uz, E);
  Q[0] += f * E[0];
  T R = ux, I = uy;
#pragma unroll
  for (int m = 1; m <= 6; m++) {
    const T fE = f * E[m];
    Q[2 * m - 1] += fE * R;
    Q[2 * m] += fE * I;
    if (m < 6) {
      const T R2 = R * ux - I * uy;
      const T I2 = R * uy + I * ux;
      R = R2;
      I = I2;
    }
  }
}

// S = w . v(u) and its gradient with respect to (ux, uy, uz) taken as free
// variables (v is a polynomial in them).  d(zeta^m)/dux = m zeta^(m-1),
// d(zeta^m)/duy = i m zeta^(m-1), dE_m/duz = rat_m E_{m+1}.
template <typename T>
__device__ __forceinline__ void grad_s(const YCoef<T>& c, T ux, T uy, T uz, const T w[13], T& S,
                                       T& Sx, T& Sy, T& Sz) {
  T E[7];
  eval_E(c, uz, E);
  S = w[0] * E[0];
  Sz = w[0] * c.rat[0] * E[1];
  Sx = T(0);
  Sy = T(0);
  T Rp = T(1), Ip = T(0), R = ux, I = uy;
#pragma unroll
  for (int m = 1; m <= 6; m++) {
    const T wa = w[2 * m - 1], wb = w[2 * m];
    const T Tm = wa * R + wb * I;
    const T U = wa * Rp + wb * Ip;
    const T V = wb * Rp - wa * Ip;
    const T mE = T(m) * E[m];
    S += E[m] * Tm;
    Sx += mE * U;
    Sy += mE * V;
    if (m < 6) {
      Sz += c.rat[m] * E[m + 1] * Tm;
      const T R2 = R * ux - I * uy;
      const T I2 = R * uy + I * ux;
      Rp = R;
      Ip = I;
      R = R2;
      I = I2;
    }
  }
}

template <typename T>
__device__ __forceinline__ void load_row16(const T* row, T v[16]) {
  const vec4_t<T>* p = reinterpret_cast<const vec4_t<T>*>(row);
#pragma unroll
  for (int q = 0; q < 4; q++) {
    vec4_t<T> x = p[q];
    v[4 * q + 0] = x.x;
    v[4 * q + 1] = x.y;
    v[4 * q + 2] = x.z;
    v[4 * q + 3] = x.w;
  }
}

template <typename T>
__device__ __forceinline__ void store_row16(T* row, const T v[16]) {
  vec4_t<T>* p = reinterpret_cast<vec4_t<T>*>(row);
#pragma unroll
  for (int q = 0; q < 4; q++) {
    vec4_t<T> x;
    x.x = v[4 * q + 0];
    x.y = v[4 * q + 1];
    x.z = v[4 * q + 2];
    x.w = v[4 * q + 3];
    p[q] = x;
  }
}

// --------------------------------------------------------------------------
// Cell list and neighbour list (every rebuild)
// --------------------------------------------------------------------------
__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

// Cell coordinates of one position, FP64 with no contraction so that the
// ids match a plain IEEE evaluation of w = x - L floor(x/L),
// c = clamp(floor(w * n/L), 0, n-1).
__device__ __forceinline__ bool cell_coords(float4 p, const CellGeom& g, int32_t c[3]) {
#pragma clang fp contract(off)
  const double x[3] = {(double)p.x, (double)p.y, (double)p.z};
  bool ok = true;
  for (int a = 0; a < 3; a++) {
    if (!isfinite(x[a])) {
      ok = false;
      c[a] = 0;
      continue;
    }
    double w = x[a] - g.L[a] * floor(x[a] / g.L[a]);
    double f = floor(w * g.inv[a]);
    f = f < 0.0 ? 0.0 : f;
    f = f > (double)(g.nc[a] - 1) ? (double)(g.nc[a] - 1) : f;
    c[a] = (int32_t)f;
  }
  return ok;
}

__global__ __launch_bounds__(kBlock) void k_cell_ids(const float4* __restrict__ pos, int64_t n,
                                                     CellGeom g, int32_t* __restrict__ cell,
                                                     int32_t* __restrict__ count, int32_t* err) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t c[3];
  if (!cell_coords(pos[i], g, c)) atomicOr(err, kErrNonFinite);
  int32_t id = (c[2] * g.nc[1] + c[1]) * g.nc[0] + c[0];
  cell[i] = id;
  atomicAdd(&count[id], 1);
}

// Exclusive prefix sum of the cell counts in one block of 1024 threads: each
// thread sums a contiguous chunk, the chunk sums are scanned in LDS, then each
// thread writes its chunk.  Also clears the scatter cursors.
__global__ __launch_bounds__(1024) void k_scan_cells(const int32_t* __restrict__ count, int64_t ncells,
                                                     int32_t* __restrict__ start, int32_t* __restrict__ fill) {
  __shared__ int32_t sums[1024];
  const int tid = threadIdx.x;
  const int64_t per = (ncells + 1023) / 1024;
  const int64_t b = tid * per;
  const int64_t e = b + per < ncells ? b + per : ncells;
  int32_t s = 0;
  for (int64_t i = b; i < e; i++) s += count[i];
  sums[tid] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int32_t v = tid >= off ? sums[tid - off] : 0;
    __syncthreads();
    sums[tid] += v;
    __syncthreads();
  }
  int32_t run = sums[tid] - s;
  for (int64_t i = b; i < e; i++) {
    start[i] = run;
    run += count[i];
    fill[i] = 0;
  }
  if (tid == 1023) start[ncells] = sums[1023];
}

__global__ __launch_bounds__(kBlock) void k_scatter(const int32_t* __restrict__ cell, int64_t n,
                                                    const int32_t* __restrict__ start,
                                                    int32_t* __restrict__ fill, int32_t* __restrict__ perm) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t c = cell[i];
  int32_t slot = atomicAdd(&fill[c], 1);
  perm[start[c] + slot] = (int32_t)i;
}

// The atomic scatter leaves each cell's atoms in arbitrary order; sorting each
// (short) segment by atom id makes the permutation the unique stable order.
__global__ __launch_bounds__(kBlock) void k_sort_cells(const int32_t* __restrict__ start, int64_t ncells,
                                                       int32_t* __restrict__ perm) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncells) return;
  const int32_t b = start[c], e = start[c + 1];
  for (int32_t i = b + 1; i < e; i++) {
    int32_t v = perm[i];
    int32_t k = i - 1;
    while (k >= b && perm[k] > v) {
      perm[k + 1] = perm[k];
      k--;
    }
    perm[k + 1] = v;
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_gather(const float4* __restrict__ pos, const int32_t* __restrict__ perm,
                                                   int64_t n, vec4_t<T>* __restrict__ pos_s, int32_t* err) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  float4 p = pos[perm[t]];
  if (!(isfinite(p.x) && isfinite(p.y) && isfinite(p.z))) atomicOr(err, kErrNonFinite);
  vec4_t<T> q;
  q.x = (T)p.x;
  q.y = (T)p.y;
  q.z = (T)p.z;
  q.w = (T)p.w;
  pos_s[t] = q;
}

// Full neighbour rows in sorted order.  The pair test is FP64 on the FP32
// coordinates, no contraction: d = x_j - x_i, d -= L rint(d/L),
// r^2 = (dx dx + dy dy) + dz dz < r_list^2.  (rint(d * (1/L)) picks the same
// image as rint(d / L) for every pair that can pass the test, since such pairs
// have |d/L| far from a half integer.)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_build_nbr(const vec4_t<T>* __restrict__ pos_s, int64_t n, CellGeom g,
                                                      double rl2, const int32_t* __restrict__ start,
                                                      int32_t* __restrict__ nbr, int32_t kmax,
                                                      int32_t* __restrict__ cnt, int32_t* err,
                                                      int32_t* maxcnt, unsigned long long* total) {
#pragma clang fp contract(off)
  __shared__ double red[kBlock / 64];
  const int64_t t = logical_block() * kBlock + threadIdx.x;
  int32_t count = 0;
  if (t < n) {
    const vec4_t<T> pi = pos_s[t];
    float4 pf;
    pf.x = (float)pi.x;
    pf.y = (float)pi.y;
    pf.z = (float)pi.z;
    pf.w = 0.f;
    int32_t c[3];
    cell_coords(pf, g, c);
    const double xi = (double)pi.x, yi = (double)pi.y, zi = (double)pi.z;
    int32_t* row = nbr + t * (int64_t)kmax;
    for (int dz = -1; dz <= 1; dz++) {
      int32_t cz = c[2] + dz;
      cz = cz < 0 ? cz + g.nc[2] : (cz >= g.nc[2] ? cz - g.nc[2] : cz);
      for (int dy = -1; dy <= 1; dy++) {
        int32_t cy = c[1] + dy;
        cy = cy < 0 ? cy + g.nc[1] : (cy >= g.nc[1] ? cy - g.nc[1] : cy);
        for (int dx = -1; dx <= 1; dx++) {
          int32_t cx = c[0] + dx;
          cx = cx < 0 ? cx + g.nc[0] : (cx >= g.nc[0] ? cx - g.nc[0] : cx);
          const int32_t cc = (cz * g.nc[1] + cy) * g.nc[0] + cx;
          const int32_t ue = start[cc + 1];
          for (int32_t u = start[cc]; u < ue; u++) {
            if (u == t) continue;
            const vec4_t<T> pj = pos_s[u];
            double d0 = (double)pj.x - xi;
            double d1 = (double)pj.y - yi;
            double d2 = (double)pj.z - zi;
            d0 = d0 - g.L[0] * rint(d0 * g.invL[0]);
            d1 = d1 - g.L[1] * rint(d1 * g.invL[1]);
            d2 = d2 - g.L[2] * rint(d2 * g.invL[2]);
            const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
            if (r2 < rl2) {
              if (count < kmax) row[count] = u;
              count++;
            }
          }
        }
      }
    }
    cnt[t] = count;
    if (count > kmax) atomicOr(err, kErrOverflow);
  }
  // block max and sum, then one atomic each per block
  int32_t m = count;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    int32_t v = __shfl_down(m, o, 64);
    m = v > m ? v : m;
  }
  double s = block_sum((double)count, red);
  __shared__ int32_t wmax[kBlock / 64];
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t bm = 0;
    for (int i = 0; i < kBlock / 64; i++) bm = wmax[i] > bm ? wmax[i] : bm;
    atomicMax(maxcnt, bm);
    atomicAdd(total, (unsigned long long)s);
  }
}

// --------------------------------------------------------------------------
// q6 crystalline count: four gather passes over the neighbour rows.
// --------------------------------------------------------------------------

// P1: Q_t = sum_j f v(r_hat), qhat_t = Q_t/|Q_t|; with CN also the per-atom
// coordination sum and its block partial.
template <typename T, bool CN>
__global__ __launch_bounds__(kBlock) void k_q6_p1(CvArgs<T> a) {
  __shared__ double red[kBlock / 64];
  const int64_t t = logical_block() * kBlock + threadIdx.x;
  double cn_part = 0.0;
  if (t < a.n) {
    const vec4_t<T> pi = a.pos_s[t];
    const int32_t c = min(a.cnt[t], a.kmax);
    const int32_t* row = a.nbr + t * (int64_t)a.kmax;
    T Q[13];
#pragma unroll
    for (int m = 0; m < 13; m++) Q[m] = T(0);
    T fsum = T(0), cnsum = T(0);
    for (int32_t k = 0; k < c; k++) {
      const vec4_t<T> pj = a.pos_s[row[k]];
      T dx, dy, dz;
      const T r2 = pair_vec(pi, pj, a, dx, dy, dz);
      if (r2 < a.rc2) {
        const T rinv = g_rsqrt(r2);
        const T r = r2 * rinv;
        T df;
        const T f = taper_w(r, a, df);
        accumulate_y(a.yc, dx * rinv, dy * rinv, dz * rinv, f, Q);
        fsum += f;
        if (CN) {
          const T x = r * a.cn_r0inv;
          const T x2 = x * x;
          cnsum += g_rcp(T(1) + x2 * x2 * x2);
        }
      }
    }
    T qq = T(0);
#pragma unroll
    for (int m = 0; m < 13; m++) qq += Q[m] * Q[m];
    const T qn = g_sqrt(qq);
    const T inv = qn >= T(1e-12) ? T(1) / qn : T(0);
    T rowv[16];
#pragma unroll
    for (int m = 0; m < 13; m++) rowv[m] = Q[m] * inv;
    rowv[13] = qn;
    rowv[14] = T(0);
    rowv[15] = fsum;
    store_row16(a.qrow + t * 16, rowv);
    if (CN) {
      a.cn_atom[t] = cnsum;
      cn_part = (double)cnsum;
    }
  }
  if (CN) {
    double b = block_sum(cn_part, red);
    if (threadIdx.x == 0) store_agent(&a.part_b[blockIdx.x], b);
  }
}

// P2: n_t = sum_j f b(qhat_t . qhat_j), c_t, c'_t; s = sum c in FP64.
template <typename T, bool CN>
__global__ __launch_bounds__(kBlock) void k_q6_p2(CvArgs<T> a) {
  __shared__ double red[kBlock / 64];
  const int64_t t = logical_block() * kBlock + threadIdx.x;
  double c_part = 0.0;
  if (t < a.n) {
    const vec4_t<T> pi = a.pos_s[t];
    T qi[16];
    load_row16(a.qrow + t * 16, qi);
    const int32_t c = min(a.cnt[t], a.kmax);
    const int32_t* row = a.nbr + t * (int64_t)a.kmax;
    T nbond = T(0);
    for (int32_t k = 0; k < c; k++) {
      const int32_t j = row[k];
      const vec4_t<T> pj = a.pos_s[j];
      T dx, dy, dz;
      const T r2 = pair_vec(pi, pj, a, dx, dy, dz);
      if (r2 < a.rc2) {
        const T r = g_sqrt(r2);
        T df;
        const T f = taper_w(r, a, df);
        T qj[16];
        load_row16(a.qrow + (int64_t)j * 16, qj);
        T d = T(0);
#pragma unroll
        for (int m = 0; m < 13; m++) d += qi[m] * qj[m];
        nbond += f * logistic((d - a.bond_d0) * a.inv_bond_w);
      }
    }
    const T cc = logistic((nbond - a.count_n0) * a.inv_count_w);
    const T dc = cc * (T(1) - cc) * a.inv_count_w;
    a.qrow[t * 16 + 14] = dc;
    a.nb[t] = nbond;
    c_part = (double)cc;
  }
  const double b = block_sum(c_part, red);
  if (threadIdx.x == 0) store_agent(&a.part_a[blockIdx.x], b);
  if (last_block_done(a.ticket)) {
    double sq = 0.0, scn = 0.0;
    for (int64_t i = threadIdx.x; i < (int64_t)gridDim.x; i += blockDim.x) {
      sq += load_agent(&a.part_a[i]);
      if (CN) scn += load_agent(&a.part_b[i]);
    }
    sq = block_sum(sq, red);
    if (CN) scn = block_sum(scn, red);
    if (threadIdx.x == 0) {
      double s0 = CN ? scn * a.inv_n : sq;
      a.s_int[0] = s0;
      if (a.s_out) a.s_out[0] = s0;
      if (CN) {
        a.s_int[1] = sq;
        if (a.s_out) a.s_out[1] = sq;
      }
      if (!isfinite(s0) || !isfinite(sq)) atomicOr(a.err, kErrNonFinite);
    }
    release_ticket(a.ticket);
  }
}

// P3: g_t = ds/dQ_t = (I - qhat qhat^T)/|Q_t| sum_j f b'(d_tj) (c'_t + c'_j) qhat_j.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_q6_p3(CvArgs<T> a) {
  const int64_t t = logical_block() * kBlock + threadIdx.x;
  if (t >= a.n) return;
  const vec4_t<T> pi = a.pos_s[t];
  T qi[16];
  load_row16(a.qrow + t * 16, qi);
  const T dci = qi[14];
  const int32_t c = min(a.cnt[t], a.kmax);
  const int32_t* row = a.nbr + t * (int64_t)a.kmax;
  T h[13];
#pragma unroll
  for (int m = 0; m < 13; m++) h[m] = T(0);
  for (int32_t k = 0; k < c; k++) {
    const int32_t j = row[k];
    const vec4_t<T> pj = a.pos_s[j];
    T dx, dy, dz;
    const T r2 = pair_vec(pi, pj, a, dx, dy, dz);
    if (r2 < a.rc2) {
      const T r = g_sqrt(r2);
      T df;
      const T f = taper_w(r, a, df);
      T qj[16];
      load_row16(a.qrow + (int64_t)j * 16, qj);
      T d = T(0);
#pragma unroll
      for (int m = 0; m < 13; m++) d += qi[m] * qj[m];
      const T b = logistic((d - a.bond_d0) * a.inv_bond_w);
      const T coef = f * b * (T(1) - b) * a.inv_bond_w * (dci + qj[14]);
#pragma unroll
      for (int m = 0; m < 13; m++) h[m] += coef * qj[m];
    }
  }
  T proj = T(0);
#pragma unroll
  for (int m = 0; m < 13; m++) proj += qi[m] * h[m];
  const T inv = qi[13] >= T(1e-12) ? T(1) / qi[13] : T(0);
  T g[16];
#pragma unroll
  for (int m = 0; m < 13; m++) g[m] = (h[m] - proj * qi[m]) * inv;
  g[13] = dci;
  g[14] = T(0);
  g[15] = T(0);
  store_row16(a.grow + t * 16, g);
}

template <typename T>
__device__ __forceinline__ void write_out(const CvArgs<T>& a, int64_t t, T gx, T gy, T gz) {
  const int32_t id = a.perm[t];
  vec4_t<T>* out = reinterpret_cast<vec4_t<T>*>(a.out4) + id;
  vec4_t<T> v = *out;
  if (a.mode == 0) {
    v.x -= gx;
    v.y -= gy;
    v.z -= gz;
  } else {
    v.x = gx;
    v.y = gy;
    v.z = gz;
  }
  *out = v;
  if (!(isfinite(v.x) && isfinite(v.y) && isfinite(v.z))) atomicOr(a.err, kErrNonFinite);
}

// P4: the chain rule onto positions, gathered per atom:
//   ds/dx_t = -sum_j [ (du/dr)(r_tj)^T (g_t + g_j) + (c'_t + c'_j) b_tj f'(r_tj) r_hat_tj ]
// with u(r) = f(r) v(r_hat) even in r, so that both ends of a pair reuse it.
// With CN, ds_CN/dx_t = -(2/N) sum_j sw'(r_tj) r_hat_tj joins in.
// G = sum_d seed_d ds_d/dx_t goes to out4 (F -= G, or grad = G).
template <typename T, bool CN>
__global__ __launch_bounds__(kBlock) void k_q6_p4(CvArgs<T> a) {
  const int64_t t = logical_block() * kBlock + threadIdx.x;
  if (t >= a.n) return;
  const T seed_q = a.seed ? (T)a.seed[a.dims - 1] : T(1);
  const T seed_cn = (CN && a.seed) ? (T)(a.seed[0] * 2.0 * a.inv_n) : T(0);
  const vec4_t<T> pi = a.pos_s[t];
  T gi[16];
  load_row16(a.grow + t * 16, gi);
  const T dci = gi[13];
  const int32_t c = min(a.cnt[t], a.kmax);
  const int32_t* row = a.nbr + t * (int64_t)a.kmax;
  T ax = T(0), ay = T(0), az = T(0);
  T cx = T(0), cy = T(0), cz = T(0);
  for (int32_t k = 0; k < c; k++) {
    const int32_t j = row[k];
    const vec4_t<T> pj = a.pos_s[j];
    T dx, dy, dz;
    const T r2 = pair_vec(pi, pj, a, dx, dy, dz);
    if (r2 < a.rc2) {
      const T rinv = g_rsqrt(r2);
      const T r = r2 * rinv;
      const T ux = dx * rinv, uy = dy * rinv, uz = dz * rinv;
      T df;
      const T f = taper_w(r, a, df);
      T gj[16];
      load_row16(a.grow + (int64_t)j * 16, gj);
      T w[13];
#pragma unroll
      for (int m = 0; m < 13; m++) w[m] = gi[m] + gj[m];
      T S, Sx, Sy, Sz;
      grad_s(a.yc, ux, uy, uz, w, S, Sx, Sy, Sz);
      const T ud = ux * Sx + uy * Sy + uz * Sz;
      const T fr = f * rinv;
      T px = fr * (Sx - ud * ux);
      T py = fr * (Sy - ud * uy);
      T pz = fr * (Sz - ud * uz);
      if (df != T(0)) {
        // taper shell only: the radial terms f' (S + (c'_t + c'_j) b_tj)
        T qi[16], qj[16];
        load_row16(a.qrow + t * 16, qi);
        load_row16(a.qrow + (int64_t)j * 16, qj);
        T d = T(0);
#pragma unroll
        for (int m = 0; m < 13; m++) d += qi[m] * qj[m];
        const T b = logistic((d - a.bond_d0) * a.inv_bond_w);
        const T rad = df * (S + (dci + gj[13]) * b);
        px += rad * ux;
        py += rad * uy;
        pz += rad * uz;
      }
      ax += px;
      ay += py;
      az += pz;
      if (CN) {
        const T x = r * a.cn_r0inv;
        const T x2 = x * x;
        const T x5 = x2 * x2 * x;
        const T den = T(1) + x5 * x;
        const T swp = T(-6) * x5 * a.cn_r0inv * g_rcp(den * den);
        cx += swp * ux;
        cy += swp * uy;
        cz += swp * uz;
      }
    }
  }
  const T gx = -(seed_q * ax + seed_cn * cx);
  const T gy = -(seed_q * ay + seed_cn * cy);
  const T gz = -(seed_q * az + seed_cn * cz);
  write_out(a, t, gx, gy, gz);
}

// --------------------------------------------------------------------------
// Coordination number alone (one forward, one force pass).
// --------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cn_fwd(CvArgs<T> a) {
  __shared__ double red[kBlock / 64];
  const int64_t t = logical_block() * kBlock + threadIdx.x;
  double part = 0.0;
  if (t < a.n) {
    const vec4_t<T> pi = a.pos_s[t];
    const int32_t c = min(a.cnt[t], a.kmax);
    const int32_t* row = a.nbr + t * (int64_t)a.kmax;
    T sum = T(0);
    for (int32_t k = 0; k < c; k++) {
      const vec4_t<T> pj = a.pos_s[row[k]];
      T dx, dy, dz;
      const T r2 = pair_vec(pi, pj, a, dx, dy, dz);
      if (r2 < a.rc2) {
        const T x2 = r2 * a.cn_r0inv * a.cn_r0inv;
        sum += g_rcp(T(1) + x2 * x2 * x2);
      }
    }
    a.cn_atom[t] = sum;
    part = (double)sum;
  }
  const double b = block_sum(part, red);
  if (threadIdx.x == 0) store_agent(&a.part_a[blockIdx.x], b);
  if (last_block_done(a.ticket)) {
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < (int64_t)gridDim.x; i += blockDim.x) s += load_agent(&a.part_a[i]);
    s = block_sum(s, red);
    if (threadIdx.x == 0) {
      s *= a.inv_n;
      a.s_int[0] = s;
      if (a.s_out) a.s_out[0] = s;
      if (!isfinite(s)) atomicOr(a.err, kErrNonFinite);
    }
    release_ticket(a.ticket);
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_cn_force(CvArgs<T> a) {
  const int64_t t = logical_block() * kBlock + threadIdx.x;
  if (t >= a.n) return;
  const T seed = (T)((a.seed ? a.seed[0] : 1.0) * 2.0 * a.inv_n);
  const vec4_t<T> pi = a.pos_s[t];
  const int32_t c = min(a.cnt[t], a.kmax);
  const int32_t* row = a.nbr + t * (int64_t)a.kmax;
  T cx = T(0), cy = T(0), cz = T(0);
  for (int32_t k = 0; k < c; k++) {
    const vec4_t<T> pj = a.pos_s[row[k]];
    T dx, dy, dz;
    const T r2 = pair_vec(pi, pj, a, dx, dy, dz);
    if (r2 < a.rc2) {
      const T rinv = g_rsqrt(r2);
      const T x = r2 * rinv * a.cn_r0inv;
      const T x2 = x * x;
      const T x5 = x2 * x2 * x;
      const T den = T(1) + x5 * x;
      const T swp = T(-6) * x5 * a.cn_r0inv * g_rcp(den * den) * rinv;
      cx += swp * dx;
      cy += swp * dy;
      cz += swp * dz;
    }
  }
  write_out(a, t, -seed * cx, -seed * cy, -seed * cz);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_atom_values(CvArgs<T> a, int what, int cv_kind, double* dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.n) return;
  double v = 0.0;
  if (what == GM_ATOM_CN) {
    v = (double)a.cn_atom[t];
  } else if (cv_kind != GM_CV_COORD) {
    if (what == GM_ATOM_Q6) {
      const double fs = (double)a.qrow[t * 16 + 15];
      v = fs > 0.0 ? sqrt(4.0 * M_PI / 13.0) * (double)a.qrow[t * 16 + 13] / fs : 0.0;
    } else if (what == GM_ATOM_NB) {
      v = (double)a.nb[t];
    } else if (what == GM_ATOM_C) {
      v = (double)logistic((a.nb[t] - a.count_n0) * a.inv_count_w);
    }
  }
  dst[a.perm[t]] = v;
}

// --------------------------------------------------------------------------
// Gaussian-hill bias (FP64): evaluation, or deposition of one hill.
// --------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_bias(BiasArgs a) {
  __shared__ double red[kBlock / 64];
  const int64_t K = *a.count;
  double s[2] = {a.s[0], a.dims > 1 ? a.s[1] : 0.0};
  double v = 0.0, g0 = 0.0, g1 = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < K; k += stride) {
    const double x0 = s[0] - a.centres[k * a.dims];
    double arg = x0 * x0 * a.inv2s2[0];
    double x1 = 0.0;
    if (a.dims > 1) {
      x1 = s[1] - a.centres[k * a.dims + 1];
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
    store_agent(&a.part[blockIdx.x * 3 + 0], v);
    store_agent(&a.part[blockIdx.x * 3 + 1], g0);
    store_agent(&a.part[blockIdx.x * 3 + 2], g1);
  }
  if (last_block_done(a.ticket)) {
    double V = 0.0, G0 = 0.0, G1 = 0.0;
    for (int64_t i = threadIdx.x; i < (int64_t)gridDim.x; i += blockDim.x) {
      V += load_agent(&a.part[i * 3 + 0]);
      G0 += load_agent(&a.part[i * 3 + 1]);
      G1 += load_agent(&a.part[i * 3 + 2]);
    }
    V = block_sum(V, red);
    G0 = block_sum(G0, red);
    if (a.dims > 1) G1 = block_sum(G1, red);
    if (threadIdx.x == 0) {
      if (!isfinite(V)) atomicOr(a.err, kErrNonFinite);
      if (a.deposit) {
        const double h = a.wt_scale == 0.0 ? a.w0 : a.w0 * exp(-V * a.wt_scale);
        if (K < a.capacity) {
          for (int d = 0; d < a.dims; d++) a.centres[K * a.dims + d] = s[d];
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
    release_ticket(a.ticket);
  }
}

// --------------------------------------------------------------------------
// Launchers
// --------------------------------------------------------------------------
static inline unsigned grid_of(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t g = grid_of(n, kBlock);
  if (g > 4096) g = 4096;
  k_fill_i32<<<(unsigned)g, kBlock, 0, st>>>(p, v, n);
  return hipGetLastError();
}

hipError_t launch_cell_ids(const float4* pos, int64_t n, const CellGeom& g, int32_t* cell, int32_t* count,
                           int32_t* err, hipStream_t st) {
  k_cell_ids<<<grid_of(n, kBlock), kBlock, 0, st>>>(pos, n, g, cell, count, err);
  return hipGetLastError();
}

hipError_t launch_scan_cells(const int32_t* count, int64_t ncells, int32_t* start, int32_t* fill,
                             hipStream_t st) {
  k_scan_cells<<<1, 1024, 0, st>>>(count, ncells, start, fill);
  return hipGetLastError();
}

hipError_t launch_scatter(const int32_t* cell, int64_t n, const int32_t* start, int32_t* fill, int32_t* perm,
                          hipStream_t st) {
  k_scatter<<<grid_of(n, kBlock), kBlock, 0, st>>>(cell, n, start, fill, perm);
  return hipGetLastError();
}

hipError_t launch_sort_cells(const int32_t* start, int64_t ncells, int32_t* perm, hipStream_t st) {
  k_sort_cells<<<grid_of(ncells, kBlock), kBlock, 0, st>>>(start, ncells, perm);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gather(const float4* pos, const int32_t* perm, int64_t n, vec4_t<T>* pos_s, int32_t* err,
                         hipStream_t st) {
  k_gather<T><<<grid_of(n, kBlock), kBlock, 0, st>>>(pos, perm, n, pos_s, err);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_build_nbr(const vec4_t<T>* pos_s, int64_t n, const CellGeom& g, double rl2,
                            const int32_t* start, int32_t* nbr, int32_t kmax, int32_t* cnt, int32_t* err,
                            int32_t* maxcnt, unsigned long long* total, hipStream_t st) {
  k_build_nbr<T><<<(unsigned)atom_blocks(n), kBlock, 0, st>>>(pos_s, n, g, rl2, start, nbr, kmax, cnt, err,
                                                               maxcnt, total);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_q6_forward(const CvArgs<T>& a, bool with_cn, hipStream_t st) {
  const unsigned g = (unsigned)atom_blocks(a.n);
  if (with_cn) {
    k_q6_p1<T, true><<<g, kBlock, 0, st>>>(a);
    k_q6_p2<T, true><<<g, kBlock, 0, st>>>(a);
  } else {
    k_q6_p1<T, false><<<g, kBlock, 0, st>>>(a);
    k_q6_p2<T, false><<<g, kBlock, 0, st>>>(a);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_q6_adjoint(const CvArgs<T>& a, hipStream_t st) {
  k_q6_p3<T><<<(unsigned)atom_blocks(a.n), kBlock, 0, st>>>(a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_q6_force(const CvArgs<T>& a, bool with_cn, hipStream_t st) {
  const unsigned g = (unsigned)atom_blocks(a.n);
  if (with_cn)
    k_q6_p4<T, true><<<g, kBlock, 0, st>>>(a);
  else
    k_q6_p4<T, false><<<g, kBlock, 0, st>>>(a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cn_forward(const CvArgs<T>& a, hipStream_t st) {
  k_cn_fwd<T><<<(unsigned)atom_blocks(a.n), kBlock, 0, st>>>(a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cn_force(const CvArgs<T>& a, hipStream_t st) {
  k_cn_force<T><<<(unsigned)atom_blocks(a.n), kBlock, 0, st>>>(a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_atom_values(const CvArgs<T>& a, int what, int cv_kind, double* dst, hipStream_t st) {
  k_atom_values<T><<<grid_of(a.n, kBlock), kBlock, 0, st>>>(a, what, cv_kind, dst);
  return hipGetLastError();
}

hipError_t launch_bias(const BiasArgs& a, int blocks, hipStream_t st) {
  k_bias<<<(unsigned)blocks, kBlock, 0, st>>>(a);
  return hipGetLastError();
}

#define GM_INSTANTIATE(T)                                                                                   \
  template hipError_t launch_gather<T>(const float4*, const int32_t*, int64_t, vec4_t<T>*, int32_t*,        \
                                       hipStream_t);                                                        \
  template hipError_t launch_build_nbr<T>(const vec4_t<T>*, int64_t, const CellGeom&, double, const int32_t*, \
                                          int32_t*, int32_t, int32_t*, int32_t*, int32_t*,                   \
                                          unsigned long long*, hipStream_t);                                 \
  template hipError_t launch_q6_forward<T>(const CvArgs<T>&, bool, hipStream_t);                             \
  template hipError_t launch_q6_adjoint<T>(const CvArgs<T>&, hipStream_t);                                   \
  template hipError_t launch_q6_force<T>(const CvArgs<T>&, bool, hipStream_t);                               \
  template hipError_t launch_cn_forward<T>(const CvArgs<T>&, hipStream_t);                                   \
  template hipError_t launch_cn_force<T>(const CvArgs<T>&, hipStream_t);                                     \
  template hipError_t launch_atom_values<T>(const CvArgs<T>&, int, int, double*, hipStream_t);

GM_INSTANTIATE(float)
GM_INSTANTIATE(double)

}  // namespace gm
