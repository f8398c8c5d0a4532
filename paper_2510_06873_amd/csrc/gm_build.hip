// Cell list, brick tables and neighbour list of libgpumetad (every rebuild).
//
// The cell list is a stable counting sort of atoms by cell id (counts ->
// exclusive scan -> atomic scatter -> per-cell sort by atom id), bit-exact
// against a plain sequential sort.  The cell grid is then cut into bricks
// that one workgroup each handles; a brick's atoms and its one-cell halo are
// addressed by "slots" in halo-cell order, which is also how the neighbour
// rows refer to neighbours (16-bit entries).
#include <string.h>

#include "gm_device.h"

namespace gm {

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

// atomicAdd(&base[key], 1) for every active lane of the wave, with one
// atomic per distinct key: atoms arrive in spatially coherent order, so a
// wave's lanes mostly share a few cells and would otherwise queue on the same
// addresses.  The lanes first find, without touching memory, the lowest lane
// holding their key (the group's leader) and their rank in the group; then
// every leader adds its group's size in one atomic instruction.  Returns the
// value the lane's own increment would have seen (equal keys take
// consecutive values in lane order).
__device__ __forceinline__ int32_t wave_count_add(int32_t* base, int32_t key) {
  const int lane = (int)(threadIdx.x & 63);
  uint64_t todo = __ballot(1);
  int leader = lane;
  int32_t rank = 0, size = 1;
  while (todo != 0) {
    const int first = __ffsll((unsigned long long)todo) - 1;
    const int32_t fk = __shfl(key, first, 64);
    const uint64_t same = __ballot(key == fk) & todo;
    if ((same >> lane) & 1ull) {
      leader = first;
      rank = (int32_t)__popcll(same & ((1ull << lane) - 1ull));
      size = (int32_t)__popcll(same);
    }
    todo &= ~same;
  }
  int32_t old = 0;
  if (lane == leader) old = atomicAdd(&base[key], size);
  return __shfl(old, leader, 64) + rank;
}

// Cell of atom i, its count, and its slot within the cell (the count it saw:
// unique per atom, in arrival order), which the scatter uses after the scan.
__device__ __forceinline__ void cell_ids_body(const float4* __restrict__ pos, int64_t n, const CellGeom& g,
                                              int32_t* __restrict__ cell, int32_t* __restrict__ count,
                                              int32_t* __restrict__ slot, int32_t* err, int64_t i) {
  if (i >= n) return;
  int32_t c[3];
  if (!cell_coords(pos[i], g, c)) atomicOr(err, kErrNonFinite);
  int32_t id = (c[2] * g.nc[1] + c[1]) * g.nc[0] + c[0];
  cell[i] = id;
  slot[i] = wave_count_add(count, id);
}

__global__ __launch_bounds__(kBlock) void k_cell_ids(const float4* __restrict__ pos, int64_t n,
                                                     CellGeom g, int32_t* __restrict__ cell,
                                                     int32_t* __restrict__ count, int32_t* __restrict__ slot,
                                                     int32_t* err) {
  cell_ids_body(pos, n, g, cell, count, slot, err, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// Exclusive prefix sum of n int32 values, out[n] = total, in three launches:
// tile sums (1024 values per workgroup), a scan of the tile sums in one
// workgroup, and the scan of each tile from its offset.  If zero != NULL it is
// cleared alongside (the scatter cursors of the cell sort).
constexpr int kScanTile = 1024;

__device__ __forceinline__ int32_t block_scan_incl(int32_t v, int32_t* lds) {
  const int tid = threadIdx.x;
  lds[tid] = v;
  __syncthreads();
  for (int off = 1; off < (int)blockDim.x; off <<= 1) {
    const int32_t u = tid >= off ? lds[tid - off] : 0;
    __syncthreads();
    lds[tid] += u;
    __syncthreads();
  }
  const int32_t r = lds[tid];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kScanTile) void k_tile_sums(const int32_t* __restrict__ in, int64_t n,
                                                         int32_t* __restrict__ sums) {
  __shared__ double red[kScanTile / 64];
  const int64_t i = (int64_t)blockIdx.x * kScanTile + threadIdx.x;
  const double v = i < n ? (double)in[i] : 0.0;
  const double t = block_sum(v, red);
  if (threadIdx.x == 0) sums[blockIdx.x] = (int32_t)t;
}

__global__ __launch_bounds__(kScanTile) void k_scan_sums(int32_t* __restrict__ sums, int64_t ntiles,
                                                         int32_t* __restrict__ out, int64_t n) {
  __shared__ int32_t lds[kScanTile];
  __shared__ int32_t total;
  int32_t carry = 0;
  for (int64_t base = 0; base < ntiles; base += kScanTile) {
    const int64_t i = base + threadIdx.x;
    const int32_t v = i < ntiles ? sums[i] : 0;
    const int32_t incl = block_scan_incl(v, lds);
    if (i < ntiles) sums[i] = carry + incl - v;
    if (threadIdx.x == kScanTile - 1) total = incl;
    __syncthreads();
    carry += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) out[n] = carry;
}

__global__ __launch_bounds__(kScanTile) void k_scan_tiles(const int32_t* __restrict__ in, int64_t n,
                                                          const int32_t* __restrict__ offs, int32_t* __restrict__ out,
                                                          int32_t* __restrict__ zero) {
  __shared__ int32_t lds[kScanTile];
  const int64_t i = (int64_t)blockIdx.x * kScanTile + threadIdx.x;
  const int32_t v = i < n ? in[i] : 0;
  const int32_t incl = block_scan_incl(v, lds);
  if (i < n) {
    out[i] = offs[blockIdx.x] + incl - v;
    if (zero) zero[i] = 0;
  }
}

// Exclusive scan of up to two short arrays (n <= kScanSmall each) in one
// workgroup: each thread sums a contiguous chunk, the chunk sums are scanned
// in LDS, and each thread writes its chunk's prefixes; out[n] = total and
// zero (if given) is cleared alongside.
constexpr int kScanSmall = 16 * kScanTile;

__device__ __forceinline__ void scan_small_one(const int32_t* __restrict__ in, int64_t n, int32_t* __restrict__ out,
                                               int32_t* __restrict__ zero, int32_t* lds) {
  const int64_t chunk = (n + kScanTile - 1) / kScanTile;  // <= kScanSmall / kScanTile
  const int64_t lo = threadIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
  // the chunk goes to registers in one batch of independent loads (a loop
  // of loads and sums waits for each load in turn)
  constexpr int kMaxChunk = kScanSmall / kScanTile;
  int32_t v[kMaxChunk];
#pragma unroll
  for (int j = 0; j < kMaxChunk; j++) v[j] = lo + j < hi ? in[lo + j] : 0;
  int32_t sum = 0;
#pragma unroll
  for (int j = 0; j < kMaxChunk; j++) sum += v[j];
  const int32_t incl = block_scan_incl(sum, lds);
  int32_t run = incl - sum;
#pragma unroll
  for (int j = 0; j < kMaxChunk; j++) {
    if (lo + j < hi) {
      out[lo + j] = run;
      if (zero) zero[lo + j] = 0;
    }
    run += v[j];
  }
  if (threadIdx.x == kScanTile - 1) out[n] = incl;
}

__global__ __launch_bounds__(kScanTile) void k_scan_small(const int32_t* __restrict__ in0, int64_t n0,
                                                          int32_t* __restrict__ out0, int32_t* __restrict__ zero0,
                                                          const int32_t* __restrict__ in1, int64_t n1,
                                                          int32_t* __restrict__ out1) {
  __shared__ int32_t lds[kScanTile];
  scan_small_one(in0, n0, out0, zero0, lds);
  if (in1) scan_small_one(in1, n1, out1, nullptr, lds);
}

// Clears what a rebuild accumulates into: the cell counts, the list
// statistics and the out-of-box flag.
__device__ __forceinline__ void reset_build_body(int32_t* __restrict__ count, int64_t ncells,
                                                 int32_t* __restrict__ stats, int32_t* __restrict__ err, int64_t i) {
  if (i < ncells) count[i] = 0;
  if (i < 4) stats[i] = 0;
  if (i == 0) err[1] = 0;
}

__global__ __launch_bounds__(kBlock) void k_reset_build(int32_t* __restrict__ count, int64_t ncells,
                                                        int32_t* __restrict__ stats, int32_t* __restrict__ err) {
  reset_build_body(count, ncells, stats, err, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

__device__ __forceinline__ void scatter_body(const int32_t* __restrict__ cell, int64_t n,
                                             const int32_t* __restrict__ start, const int32_t* __restrict__ slot,
                                             int32_t* __restrict__ scat, int64_t i) {
  if (i >= n) return;
  scat[start[cell[i]] + slot[i]] = (int32_t)i;
}

__global__ __launch_bounds__(kBlock) void k_scatter(const int32_t* __restrict__ cell, int64_t n,
                                                    const int32_t* __restrict__ start,
                                                    const int32_t* __restrict__ slot, int32_t* __restrict__ scat) {
  scatter_body(cell, n, start, slot, scat, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// The scatter leaves each cell's atoms in arrival order; placing each
// atom at its rank by id within its cell's segment makes the permutation the
// unique stable order.  One thread per atom counts the smaller ids of its
// segment (the segment's reads are shared by its atoms and cached), so dense
// cells cost linear time per atom instead of a quadratic sort per cell.
__device__ __forceinline__ void rank_cells_body(const int32_t* __restrict__ cell, const int32_t* __restrict__ start,
                                                const int32_t* __restrict__ scattered, int64_t n,
                                                int32_t* __restrict__ perm, int64_t t) {
  if (t >= n) return;
  const int32_t v = scattered[t];
  const int32_t c = cell[v];
  const int32_t b = start[c], e = start[c + 1];
  int32_t r = 0;
  for (int32_t k = b; k < e; k++) r += scattered[k] < v ? 1 : 0;
  perm[b + r] = v;
}

__global__ __launch_bounds__(kBlock) void k_rank_cells(const int32_t* __restrict__ cell,
                                                       const int32_t* __restrict__ start,
                                                       const int32_t* __restrict__ scattered, int64_t n,
                                                       int32_t* __restrict__ perm) {
  rank_cells_body(cell, start, scattered, n, perm, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

template <typename T>
__device__ __forceinline__ void gather_body(const GatherArgs& a, int64_t t) {
  if (t >= a.n) return;
  const float4 p = a.pos[a.perm[t]];
  if (!(isfinite(p.x) && isfinite(p.y) && isfinite(p.z))) atomicOr(a.err, kErrNonFinite);
  // A coordinate outside [0, L) may sit in a cell of another image: the CV
  // passes then take the minimum image for every pair until the next rebuild
  // clears the flag (one atomic per wave).
  const bool out = !(p.x >= 0.f && p.x < a.L[0] && p.y >= 0.f && p.y < a.L[1] && p.z >= 0.f && p.z < a.L[2]);
  const uint64_t m = __ballot(out);
  if (m != 0 && (int)(threadIdx.x & 63) == __ffsll((unsigned long long)m) - 1) atomicOr(a.err + 1, 1);
  vec4_t<T> q;
  q.x = (T)p.x;
  q.y = (T)p.y;
  q.z = (T)p.z;
  q.w = (T)p.w;
  reinterpret_cast<vec4_t<T>*>(a.pos_s)[t] = q;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_gather(GatherArgs a) {
  gather_body<T>(a, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_gather_batch(const GatherArgs* __restrict__ tab,
                                                         const int32_t* __restrict__ blk_start, int32_t W) {
  const int64_t g = blockIdx.x;
  int32_t lo = 0, hi = W;
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (blk_start[mid] <= g) lo = mid; else hi = mid;
  }
  gather_body<T>(tab[lo], (g - blk_start[lo]) * blockDim.x + threadIdx.x);
}

// Inclusive prefix sum of v over the workgroup's threads in thread order
// (blockDim.x a multiple of 64, at most kBlock): shuffle scans within each
// wave, then each wave adds the totals of the waves before it.  All threads
// call; wsum holds kBlock / 64 ints of LDS.
__device__ __forceinline__ int32_t block_scan_incl_wave(int32_t v, int32_t* wsum) {
  const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t u = __shfl_up(v, o, 64);
    if (lane >= o) v += u;
  }
  if (lane == 63) wsum[w] = v;
  __syncthreads();
  int32_t add = 0;
  for (int i = 0; i < w; i++) add += wsum[i];
  __syncthreads();
  return v + add;
}

// --------------------------------------------------------------------------
// Bricks: halo sizes, halo slot tables, owned atoms (every rebuild)
// --------------------------------------------------------------------------
// One wave per brick: lanes over the halo cells, wave sums of the halo and
// owned atom counts.
__device__ __forceinline__ void brick_count_body(const int32_t* __restrict__ start, const BrickGeom& g,
                                                 int32_t* __restrict__ H, int32_t* __restrict__ O, int64_t blk) {
  const int64_t b = blk * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (b >= g.nbricks) return;
  const BrickShape s = brick_shape(b, g);
  const int nh = s.h[0] * s.h[1] * s.h[2];
  int32_t h = 0, own = 0;
  for (int i = lane; i < nh; i += 64) {
    const int hx = i % s.h[0], hy = (i / s.h[0]) % s.h[1], hz = i / (s.h[0] * s.h[1]);
    const int32_t c = halo_cell_id(s, g, hx, hy, hz);
    const int32_t k = start[c + 1] - start[c];
    h += k;
    if (hx >= 1 && hx <= s.e[0] && hy >= 1 && hy <= s.e[1] && hz >= 1 && hz <= s.e[2]) own += k;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    h += __shfl_down(h, o, 64);
    own += __shfl_down(own, o, 64);
  }
  if (lane == 0) {
    H[b] = h;
    O[b] = own;
  }
}

__global__ __launch_bounds__(kBlock) void k_brick_count(const int32_t* __restrict__ start, BrickGeom g,
                                                        int32_t* __restrict__ H, int32_t* __restrict__ O) {
  brick_count_body(start, g, H, O, blockIdx.x);
}

// One workgroup per brick: slot prefix over the halo cells, the sorted
// position of every halo slot, and for every owned atom its slot, sorted
// position and own halo cell.
__device__ __forceinline__ void brick_fill_body(const int32_t* __restrict__ start, const BrickGeom& g,
                                                const BrickIndex& bi, int32_t* __restrict__ hp_out,
                                                int32_t* __restrict__ halo_rank, int32_t* __restrict__ owned_slot,
                                                int32_t* __restrict__ owned_rank, int32_t* __restrict__ owned_hcell,
                                                int32_t* err, int64_t b) {
  static_assert(kHaloCells <= kBlock && kOwnCells <= kBlock, "one thread per halo cell");
  __shared__ int32_t hcell[kHaloCells], hpre[kHaloCells + 1];
  __shared__ int32_t oh[kOwnCells], opre[kOwnCells + 1];
  __shared__ int32_t wsum[kBlock / 64];
  const BrickShape s = brick_shape(b, g);
  const int nh = s.h[0] * s.h[1] * s.h[2];
  const int no = s.e[0] * s.e[1] * s.e[2];
  const int t = (int)threadIdx.x;
  // thread t: halo cell t (its atom count) and owned cell t
  int32_t ch = 0;
  if (t < nh) {
    const int hx = t % s.h[0], hy = (t / s.h[0]) % s.h[1], hz = t / (s.h[0] * s.h[1]);
    const int32_t c = halo_cell_id(s, g, hx, hy, hz);
    hcell[t] = c;
    ch = start[c + 1] - start[c];
  }
  if (t < no) {
    const int ox = t % s.e[0], oy = (t / s.e[0]) % s.e[1], oz = t / (s.e[0] * s.e[1]);
    oh[t] = ((oz + 1) * s.h[1] + (oy + 1)) * s.h[0] + (ox + 1);
  }
  const int32_t hin = block_scan_incl_wave(ch, wsum);
  if (t < nh) hpre[t + 1] = hin;
  if (t == 0) hpre[0] = 0;
  __syncthreads();
  const int32_t co = t < no ? hpre[oh[t] + 1] - hpre[oh[t]] : 0;
  const int32_t oin = block_scan_incl_wave(co, wsum);
  if (t < no) opre[t + 1] = oin;
  if (t == 0) {
    opre[0] = 0;
    if (hpre[nh] > 65535) atomicOr(err, kErrOverflow);  // slots must fit 16 bits
  }
  __syncthreads();
  int32_t* hp = hp_out + b * (kHaloCells + 1);
  for (int h = threadIdx.x; h <= nh; h += blockDim.x) hp[h] = hpre[h];
  // thread t writes the slots of halo cell t, then of owned cell t (each cell's
  // atoms are consecutive in sorted order from start[cell])
  const int32_t hb = bi.hb[b];
  if (t < nh) {
    const int32_t s0 = start[hcell[t]], base = hb + hpre[t];
    for (int32_t j = 0; j < ch; j++) halo_rank[base + j] = s0 + j;
  }
  const int32_t ob = bi.ob[b];
  if (t < no) {
    const int h = oh[t];
    const int32_t s0 = start[hcell[h]], slot0 = hpre[h], base = ob + opre[t];
    for (int32_t j = 0; j < co; j++) {
      owned_slot[base + j] = slot0 + j;
      owned_rank[base + j] = s0 + j;
      owned_hcell[base + j] = h;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_brick_fill(const int32_t* __restrict__ start, BrickGeom g, BrickIndex bi,
                                                       int32_t* __restrict__ hp_out, int32_t* __restrict__ halo_rank,
                                                       int32_t* __restrict__ owned_slot, int32_t* __restrict__ owned_rank,
                                                       int32_t* __restrict__ owned_hcell, int32_t* err) {
  brick_fill_body(start, g, bi, hp_out, halo_rank, owned_slot, owned_rank, owned_hcell, err, blockIdx.x);
}

// Full neighbour rows as halo slots.  The decision is the FP64 test on the
// FP32 coordinates, no contraction: d = x_j - x_i, d -= L rint(d/L),
// r^2 = (dx dx + dy dy) + dz dz < r_list^2.  (rint(d * (1/L)) picks the same
// image as rint(d / L) for every pair that can pass the test, since such pairs
// have |d/L| far from a half integer.)  It is taken in FP32 first: r^2 in
// FP32 is within 4e-7 (relative) of the FP64 value (pair difference, three
// squares and two sums, each rounded once), so outside a band of 4e-6 around
// r_list^2 the FP32 answer is the FP64 one, and only pairs inside the band
// are tested in FP64.  The bound needs coordinates inside [0, L) (then the
// minimum image rounds once, at the pair's magnitude); if the gather flagged
// any outside, every pair takes the FP64 test.  Candidates are the atoms of
// the 27 cells around the atom's own cell: nine runs of three x-adjacent halo
// cells, whose slots are contiguous, visited in a fixed order.
//
// A group of kBuildGroup lanes builds one atom's row: it tests kBuildGroup
// consecutive candidates of a run at once, and a ballot gives each lane that
// passes the number of passing lanes before it, i.e. its entry index.  The
// row therefore holds the candidates in run order and slot order within a
// run, the order of a sequential scan.  Entry e lives in sub-row e % tpa at
// index e / tpa; the rest of each sub-row's last 16-byte piece is zeroed,
// since the CV passes read rows in whole pieces.
// MODE 0: FP32 plain differences (halo off the faces), 1: FP32 minimum image,
// 2: FP64 only (coordinates outside the box).  STAGED: every halo slot of the
// brick is in LDS (no per-candidate check for slots read from global memory).
template <int MODE, bool STAGED, typename T>
__device__ __forceinline__ void build_rows(const vec4_t<T>* __restrict__ pos_s, const CellGeom& cg,
                                           const BrickGeom& g, const BrickIndex& bi, double rl2, uint16_t* nbr,
                                           int32_t kmax, int32_t* cnt, int32_t* err, const float4* hpos,
                                           const int32_t* hp, int32_t hb, int32_t ob, int32_t O, int32_t k0,
                                           int32_t k1,
                                           int32_t hx, int32_t hxy, uint32_t wmask, int32_t& mymax, double& mysum) {
#pragma clang fp contract(off)
  float Lf[3], iLf[3], Llo[3];
#pragma unroll
  for (int d = 0; d < 3; d++) {
    Lf[d] = (float)cg.L[d];
    iLf[d] = (float)cg.invL[d];
    Llo[d] = (float)(cg.L[d] - (double)Lf[d]);
  }
  const float lo2 = (float)(rl2 * (1.0 - 4e-6)), hi2 = (float)(rl2 * (1.0 + 4e-6));
  const int lane = (int)(threadIdx.x & 63);
  const int lig = lane & (kBuildGroup - 1);
  const int gshift = lane - lig;                  // the group's first lane
  const uint32_t below = (1u << lig) - 1u;        // lanes of the group before this one
  const int32_t groups = (int32_t)(blockDim.x / kBuildGroup);
  const int32_t tsh = g.tpa == 4 ? 2 : (g.tpa == 2 ? 1 : 0);
  const int32_t cap = g.build_cap;
  for (int32_t k = k0 + (int32_t)(threadIdx.x / kBuildGroup); k < k1; k += groups) {
    const int32_t si = bi.owned_slot[ob + k];
    const int32_t hc = bi.owned_hcell[ob + k];
    float4 pi;
    if (si < cap) {
      pi = hpos[si];
    } else {
      const vec4_t<T> p = pos_s[bi.halo_rank[hb + si]];
      pi = make_float4((float)p.x, (float)p.y, (float)p.z, 0.f);
    }
    int32_t count = 0;  // the same in every lane of the group
    // entry e goes to sub-row e % TPA at index x = e / TPA: piece x / 8 of
    // that sub-row, pieces pstride8 entries apart (32-bit offsets from the
    // brick's first piece)
    uint16_t* const brow = nbr + row_first(g, ob, 0, 0);
    const uint32_t row0 = (uint32_t)(k * g.tpa * 8);
    const uint32_t pstride8 = (uint32_t)(piece_stride(g, O) * 8);
    const uint32_t pmask = (uint32_t)(g.tpa - 1);
    for (int cz = -1; cz <= 1; cz++)
      for (int cy = -1; cy <= 1; cy++) {
        const int h = hc + cz * hxy + cy * hx;  // middle cell of the x-run
        const int32_t se = hp[h + 2];
        for (int32_t base = hp[h - 1]; base < se; base += kBuildGroup) {
          const int32_t sl = base + lig;
          bool in = false;
          if (sl < se && sl != si) {
            // staged slots (nearly all) read LDS; the rest global memory
            float4 pj;
            if constexpr (STAGED) {
              pj = hpos[sl];
            } else {
              pj = hpos[min(sl, cap - 1)];
              if (sl >= cap) {
                const vec4_t<T> p = pos_s[bi.halo_rank[hb + sl]];
                pj = make_float4((float)p.x, (float)p.y, (float)p.z, 0.f);
              }
            }
            float ex, ey, ez;
            if constexpr (MODE == 1) {
              // the minimum image on the axes whose halo reaches a face; on
              // the others it is the plain difference (k = 0 in mic)
              ex = (wmask & 1u) ? mic(pj.x, pi.x, Lf[0], iLf[0], Llo[0]) : pj.x - pi.x;
              ey = (wmask & 2u) ? mic(pj.y, pi.y, Lf[1], iLf[1], Llo[1]) : pj.y - pi.y;
              ez = (wmask & 4u) ? mic(pj.z, pi.z, Lf[2], iLf[2], Llo[2]) : pj.z - pi.z;
            } else {
              ex = pj.x - pi.x;
              ey = pj.y - pi.y;
              ez = pj.z - pi.z;
            }
            const float r2f = (ex * ex + ey * ey) + ez * ez;
            in = MODE != 2 && r2f < lo2;
            if (MODE == 2 || (!in && r2f <= hi2)) {
              double d0 = (double)pj.x - (double)pi.x;
              double d1 = (double)pj.y - (double)pi.y;
              double d2 = (double)pj.z - (double)pi.z;
              d0 = d0 - cg.L[0] * rint(d0 * cg.invL[0]);
              d1 = d1 - cg.L[1] * rint(d1 * cg.invL[1]);
              d2 = d2 - cg.L[2] * rint(d2 * cg.invL[2]);
              in = d0 * d0 + d1 * d1 + d2 * d2 < rl2;
            }
          }
          // the group's ballot bits
          const uint32_t m8 = (uint32_t)(__ballot(in) >> gshift) & ((1u << kBuildGroup) - 1u);
          if (in) {
            const int32_t e = count + __popc(m8 & below);
            if (e < kmax) {
              const uint32_t x = (uint32_t)e >> tsh;
              // piece index and stride below 2^24: the full-rate 24-bit multiply
              brow[row0 + ((uint32_t)e & pmask) * 8u + __umul24(x >> 3, pstride8) + (x & 7u)] =
                  (uint16_t)sl;
            }
          }
          count += __popc(m8);
        }
      }
    const int32_t stored = count < kmax ? count : kmax;
    for (int32_t i = lig; i < 8 * g.tpa; i += kBuildGroup) {
      const int32_t part = i >> 3;
      const int32_t np = stored > part ? ((stored - 1 - part) >> tsh) + 1 : 0;
      const int32_t at = np + (i & 7);
      if (at < ((np + 7) & ~7)) nbr[row_entry(g, ob, O, k, part, at)] = 0;
    }
    if (lig == 0) {
      cnt[ob + k] = count;
      if (count > kmax) atomicOr(err, kErrOverflow);
      mymax = count > mymax ? count : mymax;
      mysum += (double)count;
    }
  }
}

// lb: the workgroup's logical index among the build_split x blocks of this
// system's launch.
template <typename T, int MAXT>
__device__ __forceinline__ void build_nbr_body(const vec4_t<T>* __restrict__ pos_s, const CellGeom& cg,
                                               const BrickGeom& g, const BrickIndex& bi, double rl2,
                                               uint16_t* __restrict__ nbr, int32_t kmax, int32_t* __restrict__ cnt,
                                               int32_t* err, int32_t* stats, int64_t lb) {
  extern __shared__ __align__(16) unsigned char smem[];
  float4* hpos = reinterpret_cast<float4*>(smem);
  __shared__ int32_t hp[kHaloCells + 1];
  __shared__ double red[MAXT / 64];
  __shared__ int32_t wmax[MAXT / 64];
  // build_split workgroups share a brick (consecutive logical indices, so on
  // one XCD): each stages the brick's halo and builds the rows of a
  // contiguous share of its owned atoms.
  const int64_t b = lb / g.build_split;
  const int32_t part = (int32_t)(lb - b * g.build_split);
  const bool live = b < g.nbricks;
  int32_t hb = 0, H = 0, ob = 0, O = 0, k0 = 0, k1 = 0, hx = 0, hxy = 0;
  int mode = 2;
  uint32_t wmask = 0;  // axes on which the halo reaches a periodic face
  if (live) {
    const BrickShape s = brick_shape(b, g);
    hx = s.h[0];
    hxy = s.h[0] * s.h[1];
    hb = bi.hb[b];
    H = bi.hb[b + 1] - hb;
    ob = bi.ob[b];
    O = bi.ob[b + 1] - ob;
    const int32_t share = (O + g.build_split - 1) / g.build_split;
    k0 = part * share < O ? part * share : O;
    k1 = k0 + share < O ? k0 + share : O;
    mode = err[1] != 0 ? 2 : (halo_touches_face(s, g) ? 1 : 0);
    for (int d = 0; d < 3; d++)
      if (s.o[d] < 2 || s.o[d] + s.e[d] > g.nc[d] - 2) wmask |= 1u << d;
    const int nh = s.h[0] * s.h[1] * s.h[2];
    for (int h = threadIdx.x; h <= nh; h += blockDim.x) hp[h] = bi.hp[b * (kHaloCells + 1) + h];
    const int32_t ns = H < g.build_cap ? H : g.build_cap;
    for (int32_t sl = threadIdx.x; sl < ns; sl += blockDim.x) {
      const vec4_t<T> p = pos_s[bi.halo_rank[hb + sl]];
      hpos[sl] = make_float4((float)p.x, (float)p.y, (float)p.z, 0.f);
    }
  }
  __syncthreads();
  int32_t mymax = 0;
  double mysum = 0.0;
  const bool staged = H <= g.build_cap;  // every halo slot in LDS
  if (mode == 0 && staged)
    build_rows<0, true, T>(pos_s, cg, g, bi, rl2, nbr, kmax, cnt, err, hpos, hp, hb, ob, O, k0, k1, hx, hxy, wmask, mymax,
                           mysum);
  else if (mode == 0)
    build_rows<0, false, T>(pos_s, cg, g, bi, rl2, nbr, kmax, cnt, err, hpos, hp, hb, ob, O, k0, k1, hx, hxy, wmask, mymax,
                            mysum);
  else if (mode == 1 && staged)
    build_rows<1, true, T>(pos_s, cg, g, bi, rl2, nbr, kmax, cnt, err, hpos, hp, hb, ob, O, k0, k1, hx, hxy, wmask, mymax,
                           mysum);
  else if (mode == 1)
    build_rows<1, false, T>(pos_s, cg, g, bi, rl2, nbr, kmax, cnt, err, hpos, hp, hb, ob, O, k0, k1, hx, hxy, wmask, mymax,
                            mysum);
  else
    build_rows<2, false, T>(pos_s, cg, g, bi, rl2, nbr, kmax, cnt, err, hpos, hp, hb, ob, O, k0, k1, hx, hxy, wmask, mymax,
                            mysum);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const int32_t v = __shfl_down(mymax, o, 64);
    mymax = v > mymax ? v : mymax;
  }
  const double bsum = block_sum(mysum, red);
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mymax;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t bm = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); i++) bm = wmax[i] > bm ? wmax[i] : bm;
    atomicMax(&stats[0], bm);
    atomicAdd(reinterpret_cast<unsigned long long*>(stats + 2), (unsigned long long)bsum);
  }
}

template <typename T, int MAXT>
__global__ __launch_bounds__(MAXT) void k_build_nbr(const vec4_t<T>* __restrict__ pos_s, CellGeom cg, BrickGeom g,
                                                      BrickIndex bi, double rl2, uint16_t* __restrict__ nbr,
                                                      int32_t kmax, int32_t* __restrict__ cnt, int32_t* err,
                                                      int32_t* stats) {
  build_nbr_body<T, MAXT>(pos_s, cg, g, bi, rl2, nbr, kmax, cnt, err, stats, logical_brick(g));
}

// --------------------------------------------------------------------------
// Rebuilds of several systems, one launch per stage: workgroup g of a stage
// serves walker w with blk[w] <= g < blk[w+1] (the stage's own prefix of
// workgroups per walker), as workgroup g - blk[w] of that walker's own launch.
// --------------------------------------------------------------------------
struct BuildSubset {
  const BuildArgs* tab[kBuildSubsetMax];
  int32_t blk[kBuildSubsetMax + 1];
  int32_t k;
};

__device__ __forceinline__ int32_t subset_walker(const BuildSubset& s, int64_t g) {
  int32_t lo = 0, hi = s.k;
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (s.blk[mid] <= g) lo = mid; else hi = mid;
  }
  return lo;
}

#define GM_SUBSET_BEGIN(s, gidx)                 \
  const int64_t g_ = (gidx);                      \
  const int32_t w_ = subset_walker((s), g_);      \
  const BuildArgs& A = *(s).tab[w_];              \
  const int64_t blk = g_ - (s).blk[w_];           \
  (void)blk;

__global__ __launch_bounds__(kBlock) void k_reset_build_b(BuildSubset s) {
  GM_SUBSET_BEGIN(s, blockIdx.x)
  reset_build_body(A.count, A.ncells, A.stats, A.err, blk * blockDim.x + threadIdx.x);
}

__global__ __launch_bounds__(kBlock) void k_cell_ids_b(BuildSubset s) {
  GM_SUBSET_BEGIN(s, blockIdx.x)
  cell_ids_body(A.ga.pos, A.n, A.cg, A.cell, A.count, A.slot, A.err, blk * blockDim.x + threadIdx.x);
}

__global__ __launch_bounds__(kScanTile) void k_scan_cells_b(BuildSubset s) {
  __shared__ int32_t lds[kScanTile];
  GM_SUBSET_BEGIN(s, blockIdx.x)
  scan_small_one(A.count, A.ncells, A.start, nullptr, lds);
}

__global__ __launch_bounds__(kBlock) void k_scatter_b(BuildSubset s) {
  GM_SUBSET_BEGIN(s, blockIdx.x)
  scatter_body(A.cell, A.n, A.start, A.slot, A.scat, blk * blockDim.x + threadIdx.x);
}

__global__ __launch_bounds__(kBlock) void k_rank_cells_b(BuildSubset s) {
  GM_SUBSET_BEGIN(s, blockIdx.x)
  rank_cells_body(A.cell, A.start, A.scat, A.n, A.perm, blk * blockDim.x + threadIdx.x);
}

__global__ __launch_bounds__(kBlock) void k_brick_count_b(BuildSubset s) {
  GM_SUBSET_BEGIN(s, blockIdx.x)
  brick_count_body(A.start, A.bg, A.brick_H, A.brick_O, blk);
}

__global__ __launch_bounds__(kScanTile) void k_scan_bricks_b(BuildSubset s) {
  __shared__ int32_t lds[kScanTile];
  GM_SUBSET_BEGIN(s, blockIdx.x)
  scan_small_one(A.brick_H, A.bg.nbricks, A.brick_hb, nullptr, lds);
  scan_small_one(A.brick_O, A.bg.nbricks, A.brick_ob, nullptr, lds);
}

__global__ __launch_bounds__(kBlock) void k_brick_fill_b(BuildSubset s) {
  GM_SUBSET_BEGIN(s, blockIdx.x)
  brick_fill_body(A.start, A.bg, A.bi, A.brick_hp, A.halo_rank, A.owned_slot, A.owned_rank, A.owned_hcell, A.err,
                  blk);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_gather_b(BuildSubset s) {
  GM_SUBSET_BEGIN(s, blockIdx.x)
  gather_body<T>(A.ga, blk * blockDim.x + threadIdx.x);
}

// The whole grid is a multiple of the XCD count (each walker's share is), so
// the XCD remap keeps a walker's bricks on few XCDs as in its own launch.
template <typename T, int MAXT>
__global__ __launch_bounds__(MAXT) void k_build_nbr_b(BuildSubset s) {
  const int64_t per = gridDim.x / kXcd;
  GM_SUBSET_BEGIN(s, ((int64_t)blockIdx.x % kXcd) * per + (int64_t)blockIdx.x / kXcd)
  build_nbr_body<T, MAXT>(reinterpret_cast<const vec4_t<T>*>(A.ga.pos_s), A.cg, A.bg, A.bi, A.rl2, A.nbr, A.kmax,
                          A.cnt, A.err, A.stats, blk);
}

// Neighbour rows as sorted positions (for inspection and tests).
__global__ __launch_bounds__(kBlock) void k_neighbor_ranks(const uint16_t* __restrict__ nbr,
                                                           const int32_t* __restrict__ cnt, BrickGeom g, BrickIndex bi,
                                                           int32_t kmax, int32_t* __restrict__ nbr_out,
                                                           int32_t* __restrict__ cnt_out) {
  const int64_t b = blockIdx.x;
  const int32_t hb = bi.hb[b], ob = bi.ob[b], O = bi.ob[b + 1] - ob;
  for (int32_t k = threadIdx.x; k < O; k += blockDim.x) {
    const int32_t r = bi.owned_rank[ob + k];
    const int32_t c = cnt[ob + k];
    const int32_t m = c < kmax ? c : kmax;
    for (int32_t e = 0; e < m; e++)
      nbr_out[(int64_t)r * kmax + e] = bi.halo_rank[hb + nbr[row_entry(g, ob, O, k, e % g.tpa, e / g.tpa)]];
    cnt_out[r] = c;
  }
}

// Sum of n int32 values into a 64-bit counter (block sums, one atomic each).
__global__ __launch_bounds__(kBlock) void k_sum_i32(const int32_t* __restrict__ v, int64_t n,
                                                    unsigned long long* out) {
  __shared__ double red[kBlock / 64];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s += (double)v[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) atomicAdd(out, (unsigned long long)s);
}

// --------------------------------------------------------------------------
// Launchers
// --------------------------------------------------------------------------
hipError_t launch_sum_i32(const int32_t* v, int64_t n, unsigned long long* out, hipStream_t st) {
  k_sum_i32<<<256, kBlock, 0, st>>>(v, n, out);
  return hipGetLastError();
}

static inline unsigned grid_of(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t g = grid_of(n, kBlock);
  if (g > 4096) g = 4096;
  k_fill_i32<<<(unsigned)g, kBlock, 0, st>>>(p, v, n);
  return hipGetLastError();
}

// A small host image copied into device memory inside the kernel arguments,
// which the runtime copies when the launch is enqueued: the host buffer may
// go away as soon as this returns, and nothing waits for the stream (a copy
// from pageable memory may).  Pieces of kUploadWords words per launch keep the
// arguments under the 4 KiB limit.
constexpr int kUploadWords = 896;
struct UploadPiece {
  uint32_t w[kUploadWords];
};

__global__ void k_upload(uint32_t* dst, UploadPiece src, int32_t n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src.w[i];
}

hipError_t launch_upload(void* dst, const void* src, size_t bytes, hipStream_t st) {
  const unsigned char* s = static_cast<const unsigned char*>(src);
  uint32_t* d = static_cast<uint32_t*>(dst);
  for (size_t off = 0; off < bytes; off += sizeof(UploadPiece)) {
    UploadPiece piece;
    const size_t nb = bytes - off < sizeof(UploadPiece) ? bytes - off : sizeof(UploadPiece);
    memset(&piece, 0, sizeof(piece));
    memcpy(piece.w, s + off, nb);
    k_upload<<<1, kBlock, 0, st>>>(d + off / 4, piece, (int32_t)((nb + 3) / 4));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_cell_ids(const float4* pos, int64_t n, const CellGeom& g, int32_t* cell, int32_t* count,
                           int32_t* slot, int32_t* err, hipStream_t st) {
  k_cell_ids<<<grid_of(n, kBlock), kBlock, 0, st>>>(pos, n, g, cell, count, slot, err);
  return hipGetLastError();
}

hipError_t launch_scan(const int32_t* in, int64_t n, int32_t* out, int32_t* zero, int32_t* tmp, hipStream_t st) {
  if (n <= kScanSmall) {
    k_scan_small<<<1, kScanTile, 0, st>>>(in, n, out, zero, nullptr, 0, nullptr);
    return hipGetLastError();
  }
  const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  k_tile_sums<<<(unsigned)ntiles, kScanTile, 0, st>>>(in, n, tmp);
  k_scan_sums<<<1, kScanTile, 0, st>>>(tmp, ntiles, out, n);
  k_scan_tiles<<<(unsigned)ntiles, kScanTile, 0, st>>>(in, n, tmp, out, zero);
  return hipGetLastError();
}

// Two exclusive scans (no zeroing); one launch when both are short.
hipError_t launch_scan2(const int32_t* in0, int32_t* out0, const int32_t* in1, int32_t* out1, int64_t n,
                        int32_t* tmp, hipStream_t st) {
  if (n <= kScanSmall) {
    k_scan_small<<<1, kScanTile, 0, st>>>(in0, n, out0, nullptr, in1, n, out1);
    return hipGetLastError();
  }
  hipError_t e = launch_scan(in0, n, out0, nullptr, tmp, st);
  return e != hipSuccess ? e : launch_scan(in1, n, out1, nullptr, tmp, st);
}

hipError_t launch_reset_build(int32_t* count, int64_t ncells, int32_t* stats, int32_t* err, hipStream_t st) {
  const int64_t n = ncells > 4 ? ncells : 4;
  k_reset_build<<<grid_of(n, kBlock), kBlock, 0, st>>>(count, ncells, stats, err);
  return hipGetLastError();
}

hipError_t launch_scatter(const int32_t* cell, int64_t n, const int32_t* start, const int32_t* slot, int32_t* scat,
                          hipStream_t st) {
  k_scatter<<<grid_of(n, kBlock), kBlock, 0, st>>>(cell, n, start, slot, scat);
  return hipGetLastError();
}

hipError_t launch_rank_cells(const int32_t* cell, const int32_t* start, const int32_t* scattered, int64_t n,
                             int32_t* perm, hipStream_t st) {
  k_rank_cells<<<grid_of(n, kBlock), kBlock, 0, st>>>(cell, start, scattered, n, perm);
  return hipGetLastError();
}

hipError_t launch_brick_count(const int32_t* start, const BrickGeom& g, int32_t* H, int32_t* O, hipStream_t st) {
  k_brick_count<<<grid_of(g.nbricks, kBlock / 64), kBlock, 0, st>>>(start, g, H, O);
  return hipGetLastError();
}

hipError_t launch_brick_fill(const int32_t* start, const BrickGeom& g, const BrickIndex& bi, int32_t* hp,
                             int32_t* halo_rank, int32_t* owned_slot, int32_t* owned_rank, int32_t* owned_hcell,
                             int32_t* err, hipStream_t st) {
  k_brick_fill<<<(unsigned)g.nbricks, kBlock, 0, st>>>(start, g, bi, hp, halo_rank, owned_slot, owned_rank,
                                                       owned_hcell, err);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gather(const GatherArgs& a, hipStream_t st) {
  k_gather<T><<<grid_of(a.n, kBlock), kBlock, 0, st>>>(a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_build_nbr(const vec4_t<T>* pos_s, const CellGeom& cg, const BrickGeom& g, const BrickIndex& bi,
                            double rl2, uint16_t* nbr, int32_t kmax, int32_t* cnt, int32_t* err, int32_t* stats,
                            hipStream_t st) {
  const size_t lds = (size_t)g.build_cap * sizeof(float4);
  const unsigned grid = (unsigned)((int64_t)g.blocks * g.build_split);
  if (g.build_threads <= kBlock)
    k_build_nbr<T, kBlock><<<grid, (unsigned)g.build_threads, lds, st>>>(pos_s, cg, g, bi, rl2, nbr, kmax, cnt, err,
                                                                         stats);
  else
    k_build_nbr<T, kBuildMaxThreads><<<grid, (unsigned)g.build_threads, lds, st>>>(pos_s, cg, g, bi, rl2, nbr, kmax,
                                                                                   cnt, err, stats);
  return hipGetLastError();
}

hipError_t launch_neighbor_ranks(const uint16_t* nbr, const int32_t* cnt, const BrickGeom& g, const BrickIndex& bi,
                                 int32_t kmax, int32_t* nbr_out, int32_t* cnt_out, hipStream_t st) {
  k_neighbor_ranks<<<(unsigned)g.nbricks, kBlock, 0, st>>>(nbr, cnt, g, bi, kmax, nbr_out, cnt_out);
  return hipGetLastError();
}

bool build_batchable(const BuildArgs& a) { return a.ncells <= kScanSmall && a.bg.nbricks <= kScanSmall; }

hipError_t launch_build_batch(const BuildArgs* const* dev, const BuildArgs* host, int32_t k, bool fp64,
                              hipStream_t st) {
  if (k < 1) return hipSuccess;
  if (k > kBuildSubsetMax) return hipErrorInvalidValue;
  BuildSubset s;
  s.k = k;
  for (int32_t w = 0; w < k; w++) s.tab[w] = dev[w];
  // workgroups per walker for a stage -> the subset's prefix; false if none
  auto prefix = [&](auto per) {
    s.blk[0] = 0;
    for (int32_t w = 0; w < k; w++) s.blk[w + 1] = s.blk[w] + (int32_t)per(host[w]);
    return s.blk[k] > 0;
  };
  const unsigned bw = kBlock / 64;  // bricks per workgroup of the brick count
  if (prefix([](const BuildArgs& a) { return grid_of(a.ncells > 4 ? a.ncells : 4, kBlock); }))
    k_reset_build_b<<<(unsigned)s.blk[k], kBlock, 0, st>>>(s);
  if (prefix([](const BuildArgs& a) { return grid_of(a.n, kBlock); })) k_cell_ids_b<<<(unsigned)s.blk[k], kBlock, 0, st>>>(s);
  if (prefix([](const BuildArgs&) { return 1; })) k_scan_cells_b<<<(unsigned)s.blk[k], kScanTile, 0, st>>>(s);
  if (prefix([](const BuildArgs& a) { return grid_of(a.n, kBlock); })) {
    k_scatter_b<<<(unsigned)s.blk[k], kBlock, 0, st>>>(s);
    k_rank_cells_b<<<(unsigned)s.blk[k], kBlock, 0, st>>>(s);
  }
  if (prefix([&](const BuildArgs& a) { return grid_of(a.bg.nbricks, (int)bw); }))
    k_brick_count_b<<<(unsigned)s.blk[k], kBlock, 0, st>>>(s);
  if (prefix([](const BuildArgs&) { return 1; })) k_scan_bricks_b<<<(unsigned)s.blk[k], kScanTile, 0, st>>>(s);
  if (prefix([](const BuildArgs& a) { return a.bg.nbricks; })) k_brick_fill_b<<<(unsigned)s.blk[k], kBlock, 0, st>>>(s);
  if (prefix([](const BuildArgs& a) { return grid_of(a.n, kBlock); })) {
    if (fp64)
      k_gather_b<double><<<(unsigned)s.blk[k], kBlock, 0, st>>>(s);
    else
      k_gather_b<float><<<(unsigned)s.blk[k], kBlock, 0, st>>>(s);
  }
  // the neighbour rows: one launch per workgroup size, with the largest
  // staging any of its walkers asks for
  for (int wide = 0; wide < 2; wide++) {
    BuildSubset u;
    u.k = 0;
    u.blk[0] = 0;
    size_t lds = 0;
    for (int32_t w = 0; w < k; w++) {
      const BrickGeom& g = host[w].bg;
      if ((g.build_threads > kBlock) != (wide == 1)) continue;
      u.tab[u.k] = dev[w];
      u.blk[u.k + 1] = u.blk[u.k] + g.blocks * g.build_split;
      u.k++;
      const size_t b = (size_t)g.build_cap * sizeof(float4);
      lds = b > lds ? b : lds;
    }
    if (u.k == 0) continue;
    const unsigned grid = (unsigned)u.blk[u.k];
    if (fp64) {
      if (wide)
        k_build_nbr_b<double, kBuildMaxThreads><<<grid, kBuildMaxThreads, lds, st>>>(u);
      else
        k_build_nbr_b<double, kBlock><<<grid, kBlock, lds, st>>>(u);
    } else {
      if (wide)
        k_build_nbr_b<float, kBuildMaxThreads><<<grid, kBuildMaxThreads, lds, st>>>(u);
      else
        k_build_nbr_b<float, kBlock><<<grid, kBlock, lds, st>>>(u);
    }
  }
  return hipGetLastError();
}

void allow_build_lds(int bytes) {
  const hipFuncAttribute A = hipFuncAttributeMaxDynamicSharedMemorySize;
  (void)hipFuncSetAttribute((const void*)k_build_nbr<float, kBlock>, A, bytes);
  (void)hipFuncSetAttribute((const void*)k_build_nbr<float, kBuildMaxThreads>, A, bytes);
  (void)hipFuncSetAttribute((const void*)k_build_nbr<double, kBlock>, A, bytes);
  (void)hipFuncSetAttribute((const void*)k_build_nbr<double, kBuildMaxThreads>, A, bytes);
  (void)hipFuncSetAttribute((const void*)k_build_nbr_b<float, kBlock>, A, bytes);
  (void)hipFuncSetAttribute((const void*)k_build_nbr_b<float, kBuildMaxThreads>, A, bytes);
  (void)hipFuncSetAttribute((const void*)k_build_nbr_b<double, kBlock>, A, bytes);
  (void)hipFuncSetAttribute((const void*)k_build_nbr_b<double, kBuildMaxThreads>, A, bytes);
  (void)hipGetLastError();
}

template <typename T>
hipError_t launch_gather_batch(const GatherArgs* tab, const int32_t* blk_start, int32_t W, int32_t blocks,
                               hipStream_t st) {
  k_gather_batch<T><<<(unsigned)blocks, kBlock, 0, st>>>(tab, blk_start, W);
  return hipGetLastError();
}
template hipError_t launch_gather_batch<float>(const GatherArgs*, const int32_t*, int32_t, int32_t, hipStream_t);
template hipError_t launch_gather_batch<double>(const GatherArgs*, const int32_t*, int32_t, int32_t, hipStream_t);
template hipError_t launch_gather<float>(const GatherArgs&, hipStream_t);
template hipError_t launch_gather<double>(const GatherArgs&, hipStream_t);
template hipError_t launch_build_nbr<float>(const float4*, const CellGeom&, const BrickGeom&, const BrickIndex&,
                                            double, uint16_t*, int32_t, int32_t*, int32_t*, int32_t*, hipStream_t);
template hipError_t launch_build_nbr<double>(const double4*, const CellGeom&, const BrickGeom&, const BrickIndex&,
                                             double, uint16_t*, int32_t, int32_t*, int32_t*, int32_t*, hipStream_t);

}  // namespace gm
