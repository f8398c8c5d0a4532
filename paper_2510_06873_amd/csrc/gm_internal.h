// Internal declarations shared by the kernels and the C-ABI layer of libgpumetad.
// gfx950 (CDNA4): 64-lane wavefronts, 256 CUs in 8 XCDs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gpumetad.h"

namespace gm {

constexpr int kBlock = 256;  // threads per block of the per-atom kernels (4 waves)
constexpr int kXcd = 8;      // workgroups are dealt to the 8 XCDs round-robin

// Sticky device error bits (read by gm_status).
constexpr int32_t kErrOverflow = 1;
constexpr int32_t kErrCapacity = 2;
constexpr int32_t kErrNonFinite = 4;

template <typename T>
struct V4;
template <>
struct V4<float> {
  using type = float4;
};
template <>
struct V4<double> {
  using type = double4;
};
template <typename T>
using vec4_t = typename V4<T>::type;

// Coefficients of E_m(z) = A_m d^m P_6/dz^m (z), the z part of the real l = 6
// harmonics (A_0 = K_0, A_m = sqrt2 (-1)^m K_m), split by parity of z, plus
// the ratios A_m / A_{m+1} that turn dE_m/dz into a multiple of E_{m+1}.
template <typename T>
struct YCoef {
  T e0[4], e1[3], e2[3], e3[2], e4[2], e5, e6;
  T rat[6];
};

// Geometry of the cell grid (FP64: the cell ids are part of the bit-exact sort).
struct CellGeom {
  double L[3];
  double inv[3];  // n_a / L_a
  double invL[3]; // 1 / L_a
  int32_t nc[3];
};

// Arguments of the per-atom CV kernels.
template <typename T>
struct CvArgs {
  const vec4_t<T>* pos_s;  // positions in sorted (cell) order
  const int32_t* nbr;      // [n][kmax] sorted positions of neighbours
  const int32_t* cnt;      // [n] true row lengths
  const int32_t* perm;     // sorted position -> caller's atom id
  int64_t n;
  int32_t kmax;
  int32_t dims;
  T L[3], invL[3], Llo[3];  // box, 1/box, and the low part of box in T
  T rc2, taper_lo, pi_over_D, half_pi_over_D;
  T bond_d0, inv_bond_w, count_n0, inv_count_w;
  T cn_r0inv;
  double inv_n;
  YCoef<T> yc;
  T* qrow;     // [n][16]: qhat(13), |Q|, c', sum f
  T* grow;     // [n][16]: g(13), c'
  T* nb;       // [n] bond counts
  T* cn_atom;  // [n] per-atom coordination sums
  double* part_a;  // per-block FP64 partial sums (count / coordination)
  double* part_b;
  unsigned* ticket;
  double* s_out;   // caller's s (dev), may equal s_int
  double* s_int;   // library copy of s
  int32_t* err;
  const double* seed;  // dV/ds or backward seed (dev double[dims]); NULL = 1
  int32_t mode;        // 0: F -= G (apply), 1: grad = G
  void* out4;          // force or gradient array [n][4] of T, caller's order
};

struct BiasArgs {
  const double* s;         // [dims]
  double* centres;         // [cap][dims]
  double* heights;         // [cap]
  int64_t* count;          // device hill count
  int64_t capacity;
  int32_t dims;
  int32_t deposit;         // 0: evaluate, 1: deposit a hill at s
  double inv2s2[2];        // 1 / (2 sigma_d^2)
  double invs2[2];         // 1 / sigma_d^2
  double w0, wt_scale;     // wt_scale = 1/(kBT (gamma-1)), 0 for plain metad
  double* part;            // [blocks][3]
  unsigned* ticket;
  double* V_out;
  double* dV_out;
  int32_t* err;
};

// ---- launchers (gm_kernels.hip) ------------------------------------------
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st);
hipError_t launch_cell_ids(const float4* pos, int64_t n, const CellGeom& g, int32_t* cell,
                           int32_t* count, int32_t* err, hipStream_t st);
hipError_t launch_scan_cells(const int32_t* count, int64_t ncells, int32_t* start, int32_t* fill,
                             hipStream_t st);
hipError_t launch_scatter(const int32_t* cell, int64_t n, const int32_t* start, int32_t* fill,
                          int32_t* perm, hipStream_t st);
hipError_t launch_sort_cells(const int32_t* start, int64_t ncells, int32_t* perm, hipStream_t st);
template <typename T>
hipError_t launch_gather(const float4* pos, const int32_t* perm, int64_t n, vec4_t<T>* pos_s,
                         int32_t* err, hipStream_t st);
template <typename T>
hipError_t launch_build_nbr(const vec4_t<T>* pos_s, int64_t n, const CellGeom& g, double rl2,
                            const int32_t* start, int32_t* nbr, int32_t kmax, int32_t* cnt,
                            int32_t* err, int32_t* maxcnt, unsigned long long* total,
                            hipStream_t st);
template <typename T>
hipError_t launch_q6_forward(const CvArgs<T>& a, bool with_cn, hipStream_t st);
template <typename T>
hipError_t launch_q6_adjoint(const CvArgs<T>& a, hipStream_t st);
template <typename T>
hipError_t launch_q6_force(const CvArgs<T>& a, bool with_cn, hipStream_t st);
template <typename T>
hipError_t launch_cn_forward(const CvArgs<T>& a, hipStream_t st);
template <typename T>
hipError_t launch_cn_force(const CvArgs<T>& a, hipStream_t st);
template <typename T>
hipError_t launch_atom_values(const CvArgs<T>& a, int what, int cv_kind, double* dst,
                              hipStream_t st);
hipError_t launch_bias(const BiasArgs& a, int blocks, hipStream_t st);

// Number of blocks launched for n atoms: a multiple of the XCD count.
inline int64_t atom_blocks(int64_t n) {
  int64_t b = (n + kBlock - 1) / kBlock;
  return ((b + kXcd - 1) / kXcd) * kXcd;
}

}  // namespace gm
