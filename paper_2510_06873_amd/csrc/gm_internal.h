// Internal declarations shared by the kernels and the C-ABI layer of libgpumetad.
// gfx950 (CDNA4): 64-lane wavefronts, 256 CUs in 8 XCDs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gpumetad.h"

namespace gm {

constexpr int kBlock = 256;  // threads per block of the per-atom kernels (4 waves)
constexpr int kBuildMaxThreads = 512;   // largest workgroup of the neighbour build
constexpr int kBuildGroup = 8;          // lanes that build one atom's row together
constexpr int kBuildFillBlocks = 1024;  // workgroups a neighbour build aims for (4 per CU)
constexpr int kBuildMaxSplit = 32;      // most workgroups sharing one brick in the build
constexpr int kXcd = 8;      // workgroups are dealt to the 8 XCDs round-robin
constexpr int32_t kMaxTorsions = 1 << 16;   // torsion forces are summed by one thread in order
constexpr int64_t kMaxFesBins = 1 << 24;
constexpr int32_t kFesNoAllocMaxBins = 1 << 16;  // bins of the allocation-free reweighting

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

// Threads per workgroup of the per-brick kernels.  FP32: 512, so that the two
// workgroups whose staged halos (78 KiB each) share a CU's 160 KiB of LDS run
// 4 waves per SIMD within 128 VGPRs.  FP64: 256 (its registers would not fit
// 4 waves per SIMD).
template <typename T>
struct BrickBlock {
  static constexpr int value = sizeof(T) == 4 ? 512 : 256;
};

// Pass 1 ranks the owned atoms of a brick by their longest in-cutoff part
// (keys clamped to kRankBins buckets); its LDS scratch after the staged
// positions: one key per thread, a histogram per wave, the bucket starts,
// then each atom's halo slot and sorted position (for the ranked records).
constexpr int kRankBins = 128;
template <typename T>
constexpr int rank_lds_bytes() {
  return (BrickBlock<T>::value * (3 + kRankBins / 64) + kRankBins) * 4;
}

// Coefficients of E_m(z) = A_m d^m P_6/dz^m (z), the z part of the real l = 6
// harmonics (A_0 = K_0, A_m = sqrt2 (-1)^m K_m), split by parity of z, plus
// the ratios A_m / A_{m+1} that turn dE_m/dz into a multiple of E_{m+1}.
template <typename T>
struct YCoef {
  T e0[4], e1[3], e2[3], e3[2], e4[2], e5, e6;  // E_m as polynomials in z^2 (times z for odd 6-m)
  T rat[6];                                     // dE_m/dz = rat_m E_{m+1}
  // The same E_m as lead_m z^(6-m mod 2) prod_k (z^2 - t_k): the roots t of
  // E_0 (3), E_1 (2), E_2 (2), E_3 (1), E_4 (1), all in (0, 1).
  T lead[5], t[9];
};

// Geometry of the cell grid (FP64: the cell ids are part of the bit-exact sort).
struct CellGeom {
  double L[3];
  double inv[3];  // n_a / L_a
  double invL[3]; // 1 / L_a
  int32_t nc[3];
};

// Brick decomposition of the cell grid.  A brick is b[0] x b[1] x b[2] cells;
// its halo adds one cell on every side (periodic).  One workgroup handles one
// brick: it stages the halo atoms in LDS ("slots", in halo-cell order), and
// neighbour entries are 16-bit slot numbers into that halo.
constexpr int kMaxBrick = 4;                                  // cells per axis
constexpr int kHaloCells = (kMaxBrick + 2) * (kMaxBrick + 2) * (kMaxBrick + 2);
constexpr int kOwnCells = kMaxBrick * kMaxBrick * kMaxBrick;

struct BrickGeom {
  int32_t nc[3];   // cells per axis
  int32_t b[3];    // brick size in cells
  int32_t nb[3];   // bricks per axis
  int32_t nbricks;
  int32_t cap;     // halo slots staged in LDS (slots beyond are read from global memory)
  int32_t blocks;  // workgroups launched per brick pass (nbricks rounded up to the XCD count)
  int32_t tpa;     // threads per owned atom (1, 2 or 4): lanes that split one atom's rows
  int32_t kpart;   // length of one part's sub-row (multiple of 8 entries, 16-byte aligned)
  int32_t build_threads;  // workgroup size of the neighbour build (kBuildGroup lanes per atom)
  int32_t build_split;    // workgroups per brick in the neighbour build (each takes a share of its atoms)
  int32_t build_cap;      // halo slots the neighbour build stages in LDS (slots beyond: global memory)
};

struct BrickIndex {
  const int32_t* hb;          // [nbricks+1] first halo slot of each brick (global numbering)
  const int32_t* ob;          // [nbricks+1] first owned atom of each brick (brick order)
  const int32_t* hp;          // [nbricks][kHaloCells+1] slot prefix over the halo cells
  const int32_t* halo_rank;   // [sum H] sorted position of each halo slot
  const int32_t* owned_slot;  // [N] halo slot of each owned atom (brick order)
  const int32_t* owned_rank;  // [N] sorted position of each owned atom
  const int32_t* owned_hcell; // [N] halo-cell index of the owned atom's own cell
};

// Arguments of the per-brick CV kernels.
template <typename T>
struct CvArgs {
  const vec4_t<T>* pos_s;  // positions in sorted (cell) order
  const uint16_t* nbr;     // neighbour slots: sub-row (owned atom, part) of kpart entries
  const int32_t* cnt;      // [N] row lengths, brick order
  uint16_t* cut;           // in-cutoff slots of the current step, same layout as nbr
  int32_t* ccnt;           // [N][tpa] in-cutoff counts per part, brick order
  int4* order;             // [N] per brick, by rank: (atom, halo slot, sorted position, 0) of the owned atoms
                           // ranked by longest in-cutoff part (pass 1)
  const int32_t* perm;     // sorted position -> caller's atom id
  BrickGeom bg;
  BrickIndex bi;
  int64_t n;
  int32_t kmax;
  int32_t dims;
  T L[3], invL[3], Llo[3];  // box, 1/box, and the low part of box in T
  T rc2, taper_lo, pi_over_D, half_pi_over_D;
  T bond_d0, inv_bond_w, count_n0, inv_count_w;
  T cn_r0inv2;  // 1/r0^2 of the coordination switch
  double inv_n;
  YCoef<T> yc;
  T* qrow;          // [N][16] by sorted position: qhat(13), |Q|, c', sum f
  T* grow;          // [N][16]: g(13), then the sum over taper pairs of (c'_i + c'_j) b_ij f'(r) r_hat (3)
  T* nb;            // [N] bond counts
  T* cn_atom;       // [N] per-atom coordination sums
  T* cn_grad;       // [N][4] per-atom coordination gradient sum_j f'(r) r_hat (w = 0)
  double* part_a;   // per-workgroup FP64 partial sums (count / coordination)
  double* part_b;
  double* s_out;    // caller's s (dev), may be NULL
  double* s_int;    // library copy of s
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
  double period[2];        // > 0: periodic dimension (nearest image of s - c)
  double* part;            // [blocks][3]
  double* V_out;
  double* dV_out;
  int32_t* err;
};

struct GatherArgs {
  const float4* pos;
  const int32_t* perm;
  int64_t n;
  void* pos_s;
  int32_t* err;  // err[0]: error bits; err[1] set when a coordinate lies outside [0, L)
  float L[3];    // box lengths
};

// Everything one walker's neighbour rebuild reads and writes, kept in device
// memory per context so that rebuilds of several walkers run as one launch per
// stage (the table entries are named by value in the launch).
struct BuildArgs {
  GatherArgs ga;  // caller positions -> sorted positions
  CellGeom cg;
  BrickGeom bg;
  BrickIndex bi;
  int64_t n, ncells;
  int32_t *cell, *count, *start, *slot, *perm, *scat, *stats, *err;
  int32_t *brick_H, *brick_O, *brick_hb, *brick_ob, *brick_hp, *halo_rank, *owned_slot, *owned_rank, *owned_hcell;
  uint16_t* nbr;
  int32_t* cnt;
  int32_t kmax;
  double rl2;
};
constexpr int kBuildSubsetMax = 64;
// Rebuilds that fit the one-workgroup scans (cells and bricks) can be batched.
bool build_batchable(const BuildArgs& a);
// Rebuild k walkers (k <= kBuildSubsetMax): dev[i] is walker i's BuildArgs in
// device memory, host[i] the same values on the host (for the grids).
hipError_t launch_build_batch(const BuildArgs* const* dev, const BuildArgs* host, int32_t k, bool fp64,
                              hipStream_t st);

// ---- launchers -------------------------------------------------------------
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st);
// Copy bytes of host memory to dst (device, at least bytes rounded up to a
// multiple of 4) through kernel arguments; src may be freed on return.
hipError_t launch_upload(void* dst, const void* src, size_t bytes, hipStream_t st);
hipError_t launch_cell_ids(const float4* pos, int64_t n, const CellGeom& g, int32_t* cell,
                           int32_t* count, int32_t* slot, int32_t* err, hipStream_t st);
// tmp: device int32[(n + 1023)/1024] scratch for the tile sums
hipError_t launch_scan(const int32_t* in, int64_t n, int32_t* out, int32_t* zero, int32_t* tmp, hipStream_t st);
hipError_t launch_scan2(const int32_t* in0, int32_t* out0, const int32_t* in1, int32_t* out1, int64_t n,
                        int32_t* tmp, hipStream_t st);
hipError_t launch_reset_build(int32_t* count, int64_t ncells, int32_t* stats, int32_t* err, hipStream_t st);
hipError_t launch_scatter(const int32_t* cell, int64_t n, const int32_t* start, const int32_t* slot,
                          int32_t* scat, hipStream_t st);
// perm[start[c] + rank] = atom: each cell's atoms of `scattered` in id order.
hipError_t launch_rank_cells(const int32_t* cell, const int32_t* start, const int32_t* scattered, int64_t n,
                             int32_t* perm, hipStream_t st);
hipError_t launch_brick_count(const int32_t* start, const BrickGeom& g, int32_t* H, int32_t* O,
                              hipStream_t st);
hipError_t launch_brick_fill(const int32_t* start, const BrickGeom& g, const BrickIndex& bi,
                             int32_t* hp, int32_t* halo_rank, int32_t* owned_slot, int32_t* owned_rank,
                             int32_t* owned_hcell, int32_t* err, hipStream_t st);
template <typename T>
hipError_t launch_gather(const GatherArgs& a, hipStream_t st);
template <typename T>
hipError_t launch_build_nbr(const vec4_t<T>* pos_s, const CellGeom& cg, const BrickGeom& g,
                            const BrickIndex& bi, double rl2, uint16_t* nbr, int32_t kmax, int32_t* cnt,
                            int32_t* err, int32_t* stats, hipStream_t st);
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
hipError_t launch_neighbor_ranks(const uint16_t* nbr, const int32_t* cnt, const BrickGeom& g,
                                 const BrickIndex& bi, int32_t kmax, int32_t* nbr_out, int32_t* cnt_out,
                                 hipStream_t st);
hipError_t launch_bias(const BiasArgs& a, int blocks, hipStream_t st);
// tab[3 w + 0..2]: the CV, bias and dV/ds buffers of walker w (2, 1, 2 doubles).
hipError_t launch_batch_values(const double* const* tab, int32_t W, double* s, double* V, double* dV, hipStream_t st);
hipError_t launch_torsions(const float4* pos, int64_t n, const int32_t* quads, int32_t count, const double* box,
                           double* phi, hipStream_t st);
hipError_t launch_torsion_forces(const float4* pos, int64_t n, const int32_t* quads, int32_t count, const double* box,
                                 const double* dV, void* force, bool fp64, hipStream_t st);
hipError_t launch_nearest(const float4* pos, int64_t n, int32_t centre, const int32_t* members, int32_t count,
                          const double* box, double* s, int32_t* atom, const double* dV, void* force, bool fp64,
                          hipStream_t st);
hipError_t launch_fes_reweight(const double* s, const double* V, int64_t T, int32_t dims, const double* lo,
                               const double* hi, const int32_t* nb, double kBT, double* F, hipStream_t st);
// The same kernels over the library's fixed per-device scratch (no allocation);
// at most kFesNoAllocMaxBins bins.
hipError_t launch_fes_reweight_noalloc(const double* s, const double* V, int64_t T, int32_t dims, const double* lo,
                                       const double* hi, const int32_t* nb, double kBT, double* F, hipStream_t st);
hipError_t launch_fes_hills(const BiasArgs& b, const double* lo, const double* hi, const int32_t* nb, double scale,
                            double* F, hipStream_t st);
void allow_fes_lds();
// Opt the staging kernels in to `bytes` of dynamic LDS.
void allow_cv_lds(int bytes);
void allow_build_lds(int bytes);
// Batched launches over many contexts ("walkers"): tab[W] device tables,
// blk_start[W+1] device prefix of the workgroups of each walker.
template <typename T>
hipError_t launch_gather_batch(const GatherArgs* tab, const int32_t* blk_start, int32_t W, int32_t blocks,
                               hipStream_t st);
// pass: 1..4 = q6 passes, 5 = coordination forward, 6 = coordination forces
template <typename T>
hipError_t launch_pass_batch(int pass, bool with_cn, bool fp_rows, const CvArgs<T>* tab, const int32_t* blk_start,
                             int32_t W, int32_t blocks, int32_t cap, hipStream_t st);
hipError_t launch_bias_batch(const BiasArgs* tab, const int32_t* blk_start, int32_t W, int32_t blocks,
                             hipStream_t st);
// Some walkers of a batch in one launch pair: device pointers to their table
// entries and the workgroup prefix, passed by value.
constexpr int kSubsetMax = 64;
struct BiasSubset {
  const BiasArgs* tab[kSubsetMax];
  int32_t blk[kSubsetMax + 1];
  int32_t k;
};
hipError_t launch_bias_subset(const BiasSubset& s, hipStream_t st);
hipError_t launch_sum_i32(const int32_t* v, int64_t n, unsigned long long* out, hipStream_t st);

// LDS bytes of one staged halo slot: position only, or position + 16-wide row.
template <typename T>
constexpr int slot_bytes(bool with_row) {
  return (int)sizeof(vec4_t<T>) * (with_row ? 5 : 1);
}

// Number of blocks launched for n atoms: a multiple of the XCD count.
inline int64_t atom_blocks(int64_t n) {
  int64_t b = (n + kBlock - 1) / kBlock;
  return ((b + kXcd - 1) / kXcd) * kXcd;
}

}  // namespace gm
