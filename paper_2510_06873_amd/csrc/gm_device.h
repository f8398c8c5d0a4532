// Device helpers shared by the kernel files of libgpumetad (gfx950).
#pragma once

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

// Minimum-image difference xj - xi - k L, k = rint((xj - xi)/L), with the
// box length split in a high part L (in T) and a low part Llo.  The image
// shift is subtracted from the coordinate that lies near the far face (xj for
// k > 0, xi for k < 0) before the two are differenced: there both operands
// are within a factor of two, so the subtraction is exact, and the result is
// rounded only at its own magnitude.  Forming xj - xi first would round a
// wrapped pair at the magnitude of L (ulp(200 A) ~ 1.5e-5 A in FP32).
template <typename T>
__device__ __forceinline__ T mic(T xj, T xi, T L, T invL, T Llo) {
  const T k = g_rint((xj - xi) * invL);
  const T a = xj - fmax(k, T(0)) * L;
  const T b = xi + fmin(k, T(0)) * L;
  return (a - b) - k * Llo;
}

// Pair vector r_j - r_i and its square.  WRAP = false is for bricks whose halo
// holds no cell on a periodic face while every coordinate lies in [0, L): no
// listed pair can then cross a face, and the plain difference is the minimum
// image.
template <bool WRAP, typename T>
__device__ __forceinline__ T pair_vec(const vec4_t<T>& pi, const vec4_t<T>& pj, const CvArgs<T>& a,
                                      T& dx, T& dy, T& dz) {
  if constexpr (WRAP) {
    dx = mic(pj.x, pi.x, a.L[0], a.invL[0], a.Llo[0]);
    dy = mic(pj.y, pi.y, a.L[1], a.invL[1], a.Llo[1]);
    dz = mic(pj.z, pi.z, a.L[2], a.invL[2], a.Llo[2]);
  } else {
    dx = pj.x - pi.x;
    dy = pj.y - pi.y;
    dz = pj.z - pi.z;
  }
  return dx * dx + dy * dy + dz * dz;
}

// Cosine-tapered q6 weight f(r) = (1 + cos(pi x))/2, x = (r - r_lo)/D on
// (r_lo, r_c), 1 below r_lo, and f'(r).
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

// FP32: with t = pi (x - 1/2), |t| <= pi/2, cos(pi x) = -sin t and
// sin(pi x) = cos t, taken from their Taylor series (through t^13 and t^12:
// truncation below 7e-9) for every pair, then selected.  The library sincos
// behind a branch costs every wave that holds one pair in the taper shell,
// which in disordered regions is nearly every wave; a wave with no lane in
// the shell (ordered regions) skips the series.
__device__ __forceinline__ float taper_w(float r, const CvArgs<float>& a, float& df) {
  constexpr double kF3 = 6.0, kF5 = kF3 * 20.0, kF7 = kF5 * 42.0, kF9 = kF7 * 72.0, kF11 = kF9 * 110.0,
                   kF13 = kF11 * 156.0;
  constexpr double kF2 = 2.0, kF4 = kF2 * 12.0, kF6 = kF4 * 30.0, kF8 = kF6 * 56.0, kF10 = kF8 * 90.0,
                   kF12 = kF10 * 132.0;
  const bool in = r > a.taper_lo;
  if (__ballot(in) == 0) {  // no lane of the wave in the taper shell
    df = 0.0f;
    return 1.0f;
  }
  const float t = fmaf(r - a.taper_lo, a.pi_over_D, -1.57079632679489662f);
  const float t2 = t * t;
  float sn = (float)(-1.0 / kF13);
  sn = fmaf(sn, t2, (float)(1.0 / kF11));
  sn = fmaf(sn, t2, (float)(-1.0 / kF9));
  sn = fmaf(sn, t2, (float)(1.0 / kF7));
  sn = fmaf(sn, t2, (float)(-1.0 / kF5));
  sn = fmaf(sn, t2, (float)(1.0 / kF3));
  sn = fmaf(sn * t2, -t, t);  // sin t
  float cs = (float)(1.0 / kF12);
  cs = fmaf(cs, t2, (float)(-1.0 / kF10));
  cs = fmaf(cs, t2, (float)(1.0 / kF8));
  cs = fmaf(cs, t2, (float)(-1.0 / kF6));
  cs = fmaf(cs, t2, (float)(1.0 / kF4));
  cs = fmaf(cs, t2, (float)(-1.0 / kF2));
  cs = fmaf(cs, t2, 1.0f);  // cos t
  df = in ? -a.half_pi_over_D * cs : 0.0f;
  return in ? fmaf(-0.5f, sn, 0.5f) : 1.0f;
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

// E_m from the roots: the products stay accurate near the zeros, where the
// power form loses digits to cancellation (about 2e-6 absolute in FP32 for
// E_0; the bond dots of pass 2 amplify that through two steep logistics).
template <typename T>
__device__ __forceinline__ void eval_E_roots(const YCoef<T>& c, T z, T E[7]) {
  const T z2 = z * z;
  E[0] = c.lead[0] * (z2 - c.t[0]) * (z2 - c.t[1]) * (z2 - c.t[2]);
  E[1] = c.lead[1] * z * (z2 - c.t[3]) * (z2 - c.t[4]);
  E[2] = c.lead[2] * (z2 - c.t[5]) * (z2 - c.t[6]);
  E[3] = c.lead[3] * z * (z2 - c.t[7]);
  E[4] = c.lead[4] * (z2 - c.t[8]);
  E[5] = z * c.e5;
  E[6] = c.e6;
}

// Q += f * v(u), v the real 13-vector of l = 6 harmonics:
// v_0 = E_0, v_{2m-1} = E_m Re (ux + i uy)^m, v_{2m} = E_m Im (ux + i uy)^m.
template <typename T>
__device__ __forceinline__ void accumulate_y(const YCoef<T>& c, T ux, T uy, T uz, T f, T Q[13]) {
  T E[7];
  eval_E_roots(c, uz, E);
  Q[0] += f * E[0];
  // (R, I) = f (ux + i uy)^m: the weight rides along the recurrence
  T R = f * ux, I = f * uy;
#pragma unroll
  for (int m = 1; m <= 6; m++) {
    Q[2 * m - 1] += E[m] * R;
    Q[2 * m] += E[m] * I;
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
  // m = 1 on its own: zeta^0 = 1, so U = w_1 and V = w_2 (no products with
  // the zero imaginary part, which IEEE rules keep the compiler from folding)
  const T T1 = w[1] * ux + w[2] * uy;
  S = w[0] * E[0] + E[1] * T1;
  Sx = E[1] * w[1];
  Sy = E[1] * w[2];
  Sz = w[0] * c.rat[0] * E[1] + c.rat[1] * E[2] * T1;
  T Rp = ux, Ip = uy;
  T R = ux * ux - uy * uy, I = ux * uy + uy * ux;
#pragma unroll
  for (int m = 2; m <= 6; m++) {
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


// Brick coordinates and cell-id helpers.
__device__ __forceinline__ int32_t wrap_cell(int32_t c, int32_t n) { return c < 0 ? c + n : (c >= n ? c - n : c); }

struct BrickShape {
  int32_t o[3];   // first cell of the brick on each axis
  int32_t e[3];   // brick extent in cells (edge bricks may be smaller)
  int32_t h[3];   // halo extent (e + 2)
};

__device__ __forceinline__ BrickShape brick_shape(int64_t b, const BrickGeom& g) {
  BrickShape s;
  int32_t ib[3];
  ib[0] = (int32_t)(b % g.nb[0]);
  ib[1] = (int32_t)((b / g.nb[0]) % g.nb[1]);
  ib[2] = (int32_t)(b / ((int64_t)g.nb[0] * g.nb[1]));
  for (int a = 0; a < 3; a++) {
    s.o[a] = ib[a] * g.b[a];
    s.e[a] = min(g.b[a], g.nc[a] - s.o[a]);
    s.h[a] = s.e[a] + 2;
  }
  return s;
}

// A brick's halo window is cells [o-1, o+e] on each axis.  If it keeps off
// cells 0 and nc-1 on every axis, its atoms sat at least one cell (more than
// half the skin) from every face at the rebuild, so while all coordinates lie
// inside the box no pair of its halo crosses a face.
__device__ __forceinline__ bool halo_touches_face(const BrickShape& s, const BrickGeom& g) {
  bool edge = false;
#pragma unroll
  for (int d = 0; d < 3; d++) edge = edge || s.o[d] < 2 || s.o[d] + s.e[d] > g.nc[d] - 2;
  return edge;
}

// Global cell id of halo cell (hx, hy, hz) of a brick (halo coordinates start at -1).
__device__ __forceinline__ int32_t halo_cell_id(const BrickShape& s, const BrickGeom& g, int hx, int hy, int hz) {
  const int32_t cx = wrap_cell(s.o[0] - 1 + hx, g.nc[0]);
  const int32_t cy = wrap_cell(s.o[1] - 1 + hy, g.nc[1]);
  const int32_t cz = wrap_cell(s.o[2] - 1 + hz, g.nc[2]);
  return (cz * g.nc[1] + cy) * g.nc[0] + cx;
}

// Logical brick of this workgroup: XCD x (= blockIdx % 8) walks a contiguous
// range of bricks, so the halos it stages overlap in its own L2.
__device__ __forceinline__ int64_t logical_brick(const BrickGeom& g) {
  const int64_t b = blockIdx.x;
  const int64_t per = gridDim.x / kXcd;
  return (b % kXcd) * per + b / kXcd;
}

// Rows of 16-bit halo slots (neighbour rows and this step's in-cutoff rows).
// Entry e of an atom's row lives in sub-row e % tpa at index e / tpa, and a
// sub-row is stored in pieces of 8 entries (16 bytes).  A brick's rows are
// piece-major: piece q of sub-row `part` of owned atom `o` is piece
// (q O + o) tpa + part of the brick's region, which starts at entry
// ob tpa kpart (ob: the brick's first owned atom, O: its owned count).  Most
// sub-rows end in their first or second piece, so the later pieces, which
// few atoms reach, lie in cache lines of their own instead of between the
// pieces every atom reads.
//
// First entry of a sub-row (its piece 0), and the distance in pieces from one
// piece of a sub-row to the next.
__device__ __forceinline__ int64_t row_first(const BrickGeom& g, int32_t ob, int32_t o, int32_t part) {
  return (int64_t)ob * g.tpa * g.kpart + ((int64_t)o * g.tpa + part) * 8;
}

__device__ __forceinline__ int32_t piece_stride(const BrickGeom& g, int32_t O) { return O * g.tpa; }

// Entry x of a sub-row.
__device__ __forceinline__ int64_t row_entry(const BrickGeom& g, int32_t ob, int32_t O, int32_t o, int32_t part,
                                             int32_t x) {
  return row_first(g, ob, o, part) + (int64_t)(x >> 3) * piece_stride(g, O) * 8 + (x & 7);
}

// Sequential reader of one sub-row of 16-bit slots: 8 entries per 16-byte
// load, entries popped from registers by funnel shifts (no dynamic register
// indexing).  All lanes pop in lockstep.  The next 8 are loaded halfway
// through the current 8, so the wait before they are used covers a load
// issued several pairs earlier (the compiler's wait at that point is for all
// outstanding loads).
struct SlotStream {
  const uint4* src;
  uint4 cur, nxt;
  int32_t n, j, ps;

  __device__ __forceinline__ void init(const uint16_t* row, int32_t count, int32_t stride) {
    src = reinterpret_cast<const uint4*>(row);
    ps = stride;
    n = count;
    j = 0;
    cur = make_uint4(0, 0, 0, 0);
    nxt = cur;
    if (n > 0) cur = src[0];
  }

  // The same, with the row's first 16 bytes already loaded.
  __device__ __forceinline__ void init_first(const uint16_t* row, int32_t count, int32_t stride, uint4 first) {
    src = reinterpret_cast<const uint4*>(row);
    ps = stride;
    n = count;
    j = 0;
    cur = first;
    nxt = first;
  }

  __device__ __forceinline__ int32_t pop() {
    const int32_t s = (int32_t)(cur.x & 0xffffu);
    cur.x = __builtin_amdgcn_alignbit(cur.y, cur.x, 16);
    cur.y = __builtin_amdgcn_alignbit(cur.z, cur.y, 16);
    cur.z = __builtin_amdgcn_alignbit(cur.w, cur.z, 16);
    cur.w = cur.w >> 16;
    j++;
    if ((j & 7) == 4 && j + 4 < n) nxt = src[((j >> 3) + 1) * ps];
    if ((j & 7) == 0) cur = nxt;
    return s;
  }
};

// Visits the first n slots of a sub-row (pieces ps apart) in order, 8 to a block: the load of
// the next block's 16 bytes is issued before the current block is visited,
// so its wait falls after 8 bodies.  The prefetch index is clamped to the
// row's last used chunk, so the load is unconditional and in bounds.  `first`
// holds the row's first 16 bytes when the caller loaded them already.
// UNROLL = true writes the 8 bodies of a block out (each guarded by the
// row's length, slots taken by constant index); a body may then also store
// to memory, whereas a store inside the rolled inner loop (with no load
// beside it) makes the compiler wait for the prefetch before that loop.
template <bool UNROLL = false, class Body>
__device__ __forceinline__ void for_slots(const uint16_t* row, int32_t n, int32_t ps, uint4 first, Body body) {
  const uint4* src = reinterpret_cast<const uint4*>(row);
  const int32_t last = (n - 1) >> 3;
  uint4 cur = first;
  for (int32_t b = 0; b < n; b += 8) {
    const uint4 nxt = src[min((b >> 3) + 1, last) * ps];
    // Settle the wait for this block's 16 bytes here (in the first block
    // they are still in flight), so that no wait inside the block can also
    // drain the prefetch behind a store the body issued.
    asm volatile("" ::"v"(cur.x), "v"(cur.y), "v"(cur.z), "v"(cur.w));
    const int32_t m = min(8, n - b);
    if constexpr (UNROLL) {
      const uint32_t w[4] = {cur.x, cur.y, cur.z, cur.w};
#pragma unroll
      for (int e = 0; e < 8; e++)
        if (e < m) body((int32_t)((w[e >> 1] >> ((e & 1) * 16)) & 0xffffu));
    } else {
      for (int32_t e = 0; e < m; e++) {
        body((int32_t)(cur.x & 0xffffu));
        cur.x = __builtin_amdgcn_alignbit(cur.y, cur.x, 16);
        cur.y = __builtin_amdgcn_alignbit(cur.z, cur.y, 16);
        cur.z = __builtin_amdgcn_alignbit(cur.w, cur.z, 16);
        cur.w = cur.w >> 16;
      }
    }
    cur = nxt;
  }
}

__device__ __forceinline__ uint4 first_chunk(const uint16_t* row, int32_t n) {
  return n > 0 ? *reinterpret_cast<const uint4*>(row) : make_uint4(0, 0, 0, 0);
}

// Appends 16-bit slots to one sub-row, 8 per 16-byte store.  The 16 bytes
// in registers are a shift register of the last 8 slots (the newest enters
// at the top, so after 8 pushes they lie in row order and are stored);
// flush() writes the partial tail, shifted down to the front with zeros
// behind it.
struct SlotWriter {
  uint4* dst;
  uint4 buf;
  int32_t n, ps;

  __device__ __forceinline__ void init(uint16_t* row, int32_t stride) {
    dst = reinterpret_cast<uint4*>(row);
    ps = stride;
    buf = make_uint4(0, 0, 0, 0);
    n = 0;
  }

  __device__ __forceinline__ void push(int32_t s) {
    buf.x = __builtin_amdgcn_alignbit(buf.y, buf.x, 16);
    buf.y = __builtin_amdgcn_alignbit(buf.z, buf.y, 16);
    buf.z = __builtin_amdgcn_alignbit(buf.w, buf.z, 16);
    buf.w = (buf.w >> 16) | ((uint32_t)s << 16);
    n++;
    if ((n & 7) == 0) dst[((n >> 3) - 1) * ps] = buf;
  }

  __device__ __forceinline__ void flush() {
    const int r = n & 7;
    if (r) {
      // the r newest slots sit in the top r entries: shift them down by
      // 8 - r entries, bringing zeros in above
      uint4 b = buf;
      for (int k = r; k < 8; k++) {
        b.x = __builtin_amdgcn_alignbit(b.y, b.x, 16);
        b.y = __builtin_amdgcn_alignbit(b.z, b.y, 16);
        b.z = __builtin_amdgcn_alignbit(b.w, b.z, 16);
        b.w = b.w >> 16;
      }
      dst[(n >> 3) * ps] = b;
    }
  }
};

}  // namespace gm
