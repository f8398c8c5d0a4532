// Collective-variable kernels of libgpumetad, one workgroup per brick.
//
// Each pass stages the brick's halo (positions, plus the 16-wide per-atom row
// the pass needs) in LDS with coalesced loads, then every thread walks the
// neighbour slots of one owned atom reading LDS only.  Pass 1 also writes the
// slots inside r_c for this step, so passes 2-4 skip the skin pairs.
//
//   pass 1  Q_i = sum_j f(r_ij) v(r_hat_ij), qhat_i = Q_i/|Q_i|; coordination sums
//   pass 2  n_i = sum_j f b(qhat_i.qhat_j), c_i, c'_i; s = sum_i c_i (FP64)
//   pass 3  g_i = ds/dQ_i and the taper radial term of ds/dx_i
//   pass 4  ds/dx_i = -sum_j [ (du/dr)(r_ij)^T (g_i + g_j) + radial ],
//           F_i -= sum_d dV/ds_d ds_d/dx_i  (or the gradient alone)
#include <type_traits>

#include "gm_device.h"

namespace gm {

struct Brick {
  int64_t b;
  int32_t hb, H, ob, O, ns;
  bool wrap;  // pairs may cross a periodic face: minimum image needed
};

template <typename T>
__device__ __forceinline__ Brick brick_begin(const CvArgs<T>& a, int64_t brick) {
  Brick k;
  k.b = brick;
  k.hb = k.H = k.ob = k.O = k.ns = 0;
  k.wrap = true;
  if (k.b < a.bg.nbricks) {
    k.hb = a.bi.hb[k.b];
    k.H = a.bi.hb[k.b + 1] - k.hb;
    k.ob = a.bi.ob[k.b];
    k.O = a.bi.ob[k.b + 1] - k.ob;
    k.ns = k.H < a.bg.cap ? k.H : a.bg.cap;
    // plain pair differences unless the halo touches a face or the gather
    // flagged a coordinate outside the box
    k.wrap = halo_touches_face(brick_shape(k.b, a.bg), a.bg) || a.err[1] != 0;
  }
  return k;
}

// Run a pass's per-atom loop in the variant for this brick: whole halo in
// LDS or not, pairs that may wrap or not.
template <typename T, class F>
__device__ __forceinline__ auto brick_variant(const CvArgs<T>& a, const Brick& k, F f) {
  using Y = std::true_type;
  using N = std::false_type;
  if (k.H <= a.bg.cap) return k.wrap ? f(Y{}, Y{}) : f(Y{}, N{});
  return k.wrap ? f(N{}, Y{}) : f(N{}, N{});
}

template <typename T>
__device__ __forceinline__ void stage_pos(const CvArgs<T>& a, const Brick& k, vec4_t<T>* lp) {
#pragma unroll 4
  for (int32_t s = threadIdx.x; s < k.ns; s += blockDim.x) lp[s] = a.pos_s[a.bi.halo_rank[k.hb + s]];
}

// LDS record of a slot: position, then the 16-wide row (4 vectors).
template <typename T>
__device__ __forceinline__ void stage_rows(const CvArgs<T>& a, const Brick& k, const T* rows, vec4_t<T>* lr) {
#pragma unroll 4
  for (int32_t s = threadIdx.x; s < k.ns; s += blockDim.x) {
    const int32_t r = a.bi.halo_rank[k.hb + s];
    const vec4_t<T>* src = reinterpret_cast<const vec4_t<T>*>(rows + (int64_t)r * 16);
    vec4_t<T>* dst = lr + 5 * s;
    dst[0] = a.pos_s[r];
    dst[1] = src[0];
    dst[2] = src[1];
    dst[3] = src[2];
    dst[4] = src[3];
  }
}

// Fetch a slot's position (and row) from LDS; slots past the staged capacity
// come from global memory.  ALL: the whole halo is staged (no fallback path).
template <bool ALL, typename T>
__device__ __forceinline__ vec4_t<T> fetch_pos(const CvArgs<T>& a, const Brick& k, const vec4_t<T>* lp, int32_t s) {
  if (ALL || s < a.bg.cap) return lp[s];
  return a.pos_s[a.bi.halo_rank[k.hb + s]];
}

template <bool ALL, typename T>
__device__ __forceinline__ void fetch_rec(const CvArgs<T>& a, const Brick& k, const vec4_t<T>* lr, const T* rows,
                                          int32_t s, vec4_t<T>& p, T v[16]) {
  if (ALL || s < a.bg.cap) {
    const vec4_t<T>* src = lr + 5 * s;
    p = src[0];
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const vec4_t<T> x = src[1 + q];
      v[4 * q + 0] = x.x;
      v[4 * q + 1] = x.y;
      v[4 * q + 2] = x.z;
      v[4 * q + 3] = x.w;
    }
  } else {
    const int32_t r = a.bi.halo_rank[k.hb + s];
    p = a.pos_s[r];
    load_row16(rows + (int64_t)r * 16, v);
  }
}

// The force (or gradient) row of atom id, whose current value v was read
// earlier by the same thread.
template <typename T>
__device__ __forceinline__ void write_out_at(const CvArgs<T>& a, int32_t id, vec4_t<T> v, T gx, T gy, T gz) {
  vec4_t<T>* out = reinterpret_cast<vec4_t<T>*>(a.out4) + id;
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

template <typename T>
__device__ __forceinline__ void write_out(const CvArgs<T>& a, int32_t rank, T gx, T gy, T gz) {
  const int32_t id = a.perm[rank];
  write_out_at(a, id, reinterpret_cast<const vec4_t<T>*>(a.out4)[id], gx, gy, gz);
}

// Fixed-order sum of the per-workgroup partials, in one workgroup (its own
// launch, so every partial is visible without fences); writes s.
// TWO: part_b holds the coordination (scaled by 1/N), part_a the q6 count.
// SCALE: one CV held in part_a that is scaled by 1/N (the coordination alone).
template <typename T, bool TWO, bool SCALE>
__device__ __forceinline__ void finish_body(const CvArgs<T>& a) {
  __shared__ double red[kBlock / 64];
  const int32_t nblk = a.bg.blocks;
  double sa = 0.0, sb = 0.0;
  // 8 strided partials per thread and round, loaded as one batch (clamped
  // indices, the extras added as zero): the same additions in the same
  // order as one partial at a time, without a memory latency per partial.
  for (int32_t base = threadIdx.x; base < nblk; base += 8 * blockDim.x) {
    double va[8], vb[8];
#pragma unroll
    for (int u = 0; u < 8; u++) {
      const int32_t i = min(base + u * (int32_t)blockDim.x, nblk - 1);
      va[u] = a.part_a[i];
      vb[u] = TWO ? a.part_b[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; u++) {
      const bool in = base + u * (int32_t)blockDim.x < nblk;
      sa += in ? va[u] : 0.0;
      if (TWO) sb += in ? vb[u] : 0.0;
    }
  }
  sa = block_sum(sa, red);
  if (TWO) sb = block_sum(sb, red);
  if (threadIdx.x == 0) {
    const double s0 = TWO ? sb * a.inv_n : (SCALE ? sa * a.inv_n : sa);
    const double s1 = TWO ? sa : 0.0;
    a.s_int[0] = s0;
    if (a.s_out) a.s_out[0] = s0;
    if (TWO) {
      a.s_int[1] = s1;
      if (a.s_out) a.s_out[1] = s1;
    }
    if (!isfinite(s0) || !isfinite(s1)) atomicOr(a.err, kErrNonFinite);
  }
}

template <typename T, bool TWO, bool SCALE>
__global__ __launch_bounds__(kBlock) void k_finish(CvArgs<T> a) {
  finish_body<T, TWO, SCALE>(a);
}

template <typename T, bool TWO, bool SCALE>
__global__ __launch_bounds__(kBlock) void k_finish_batch(const CvArgs<T>* __restrict__ tab) {
  finish_body<T, TWO, SCALE>(tab[blockIdx.x]);
}

// Threads per atom: TPA adjacent lanes share one owned atom; lane part p
// walks the atom's rows at entries p, p + TPA, ...  (the per-step cutoff rows
// are stored as TPA interleaved sub-lists, one per part), and the parts'
// partial sums are combined with xor exchanges inside each quad of lanes
// (same result in every part).  The exchanges are DPP quad permutations, a
// register move, rather than a shuffle through the LDS crossbar; the lanes of
// one atom are active together, so every source lane holds its partial.
template <int CTRL>
__device__ __forceinline__ int32_t quad_xor(int32_t v) {
  return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xf, 0xf, false);
}

template <int CTRL>
__device__ __forceinline__ float quad_xor(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), CTRL, 0xf, 0xf, false));
}

template <int CTRL>
__device__ __forceinline__ double quad_xor(double v) {
  const int64_t b = __double_as_longlong(v);
  const int32_t lo = (int32_t)b, hi = (int32_t)(b >> 32);
  const int32_t l2 = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xf, 0xf, false);
  const int32_t h2 = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xf, 0xf, false);
  return __longlong_as_double((int64_t)(((uint64_t)(uint32_t)h2 << 32) | (uint32_t)l2));
}

// quad_perm selectors: lane q of a quad reads lane q ^ 1, respectively q ^ 2
constexpr int kQuadXor1 = 1 | (0 << 2) | (3 << 4) | (2 << 6);
constexpr int kQuadXor2 = 2 | (3 << 2) | (0 << 4) | (1 << 6);

template <typename T>
__device__ __forceinline__ T group_sum(T v, int TPA) {
  if (TPA >= 2) v += quad_xor<kQuadXor1>(v);
  if (TPA >= 4) v += quad_xor<kQuadXor2>(v);
  return v;
}

// Walk the n cutoff slots of one part, two records in flight: the next
// record is fetched before the current one is used; slot numbers come from a
// register stream over the part's sub-row.  When every slot is staged (ALL)
// the pops and LDS fetches are unconditional (only the bodies are guarded),
// so that the compiler can count the LDS reads in flight and wait for the
// current record only; past the row's end the stream yields slots of the same
// row (its zero padding or an earlier 16 bytes again), which are valid
// records.  Otherwise a fetch may go to global memory and stays guarded.
template <bool ALL, typename T, class Body>
__device__ __forceinline__ void walk_records(const CvArgs<T>& a, const Brick& k, const vec4_t<T>* lr, const T* rows,
                                             const uint16_t* crow, int32_t n, int32_t ps, uint4 first, Body body) {
  if (n <= 0) return;
  vec4_t<T> pa, pb;
  T va[16], vb[16];
  if constexpr (ALL) {
    // blocks of 8 slots, written out: slot e of a block by constant index,
    // the next block's 16 bytes loaded at the block start (its first slot is
    // the lookahead of the block's last pair)
    const uint4* src = reinterpret_cast<const uint4*>(crow);
    const int32_t last = (n - 1) >> 3;
    uint4 cur = first;
    fetch_rec<ALL>(a, k, lr, rows, (int32_t)(cur.x & 0xffffu), pa, va);
    for (int32_t b = 0; b < n; b += 8) {
      const uint4 nxt = src[min((b >> 3) + 1, last) * ps];
      const uint32_t w[4] = {cur.x, cur.y, cur.z, cur.w};
#pragma unroll
      for (int e = 0; e < 8; e += 2) {
        fetch_rec<ALL>(a, k, lr, rows, (int32_t)(w[e >> 1] >> 16), pb, vb);
        if (b + e < n) body(pa, va);
        const int32_t s2 = e + 2 < 8 ? (int32_t)(w[(e + 2) >> 1] & 0xffffu) : (int32_t)(nxt.x & 0xffffu);
        fetch_rec<ALL>(a, k, lr, rows, s2, pa, va);
        if (b + e + 1 < n) body(pb, vb);
      }
      cur = nxt;
    }
  } else {
    SlotStream st;
    st.init_first(crow, n, ps, first);
    fetch_rec<ALL>(a, k, lr, rows, st.pop(), pa, va);
    for (int32_t j = 0; j < n; j += 2) {
      const bool b_ok = j + 1 < n;
      if (b_ok) fetch_rec<ALL>(a, k, lr, rows, st.pop(), pb, vb);
      body(pa, va);
      if (b_ok) {
        if (j + 2 < n) fetch_rec<ALL>(a, k, lr, rows, st.pop(), pa, va);
        body(pb, vb);
      }
    }
  }
}

// Owned atoms of this workgroup's brick: thread -> (atom o, part), in cell
// order (pass 1) or in the order pass 1 ranked them by their longest
// in-cutoff part (passes 2-4), so that the lanes of a wave walk rows of
// similar length (a wave loops as long as its longest lane).
// TPA is a power of two: atom and part come from shifts and masks.
#define GM_FOR_OWNED(a, k)                                             \
  const int TPA = (a).bg.tpa;                                          \
  const int TSH = __builtin_ctz((unsigned)TPA);                        \
  const int32_t part = threadIdx.x & (TPA - 1);                        \
  for (int32_t o = (int32_t)(threadIdx.x >> TSH); o < (k).O; o += (int32_t)(blockDim.x >> TSH))

// The head of an owned atom in the ranked passes: its record from pass 1
// (atom, halo slot, sorted position), its in-cutoff count and the first 16
// bytes of its cut sub-row.  A thread's first head is loaded around the halo
// staging (record before, the rest after) so that these dependent loads wait
// alongside the staging instead of after it; later heads (bricks with more
// atoms than threads) are loaded in place.
struct AtomHead {
  int32_t o, si, ri, nc;
  uint4 c0;
};

template <typename T>
__device__ __forceinline__ void head_record(const CvArgs<T>& a, const Brick& k, int32_t r, AtomHead& h) {
  const int4 rec = a.order[k.ob + r];
  h.o = rec.x;
  h.si = rec.y;
  h.ri = rec.z;
}

template <typename T>
__device__ __forceinline__ void head_rows(const CvArgs<T>& a, const Brick& k, int32_t part, AtomHead& h) {
  h.nc = a.ccnt[(int64_t)(k.ob + h.o) * a.bg.tpa + part];
  h.c0 = *reinterpret_cast<const uint4*>(a.cut + row_first(a.bg, k.ob, h.o, part));  // allocated even when nc = 0
}

// Threads past the brick's atoms load the last atom's head (valid memory,
// never used), so that the loads need no branch.
template <typename T>
__device__ __forceinline__ AtomHead head_begin(const CvArgs<T>& a, const Brick& k) {
  AtomHead h;
  h.o = 0;
  h.si = h.ri = h.nc = 0;
  h.c0 = make_uint4(0, 0, 0, 0);
  if (k.O > 0) {
    const int32_t r = (int32_t)(threadIdx.x >> __builtin_ctz((unsigned)a.bg.tpa));
    head_record(a, k, r < k.O ? r : k.O - 1, h);
  }
  return h;
}

template <typename T>
__device__ __forceinline__ void head_end(const CvArgs<T>& a, const Brick& k, AtomHead& h) {
  if (k.O > 0) head_rows(a, k, (int32_t)(threadIdx.x & (a.bg.tpa - 1)), h);
}

// h starts as the thread's first head; later atoms overwrite it in place.
#define GM_FOR_RANKED(a, k, h0)                                                                \
  const int TPA = (a).bg.tpa;                                                                  \
  const int TSH = __builtin_ctz((unsigned)TPA);                                                \
  const int32_t part = threadIdx.x & (TPA - 1);                                                \
  AtomHead h = (h0);                                                                           \
  for (int32_t r_ = (int32_t)(threadIdx.x >> TSH); r_ < (k).O; r_ += (int32_t)(blockDim.x >> TSH)) \
    if ((r_ == (int32_t)(threadIdx.x >> TSH) ? (void)0 : (head_record(a, k, r_, h), head_rows(a, k, part, h))), true) \
      if (const int32_t o = h.o, si = h.si, ri = h.ri, nc = h.nc; true)

// Stable counting sort of the owned atoms by key, descending (equal keys keep
// cell order), written as order[rank] = atom.  Thread t ranks atom t: per-wave
// histograms in LDS, their prefix over waves and the bucket starts, then the
// rank among equal keys in the wave from ballots over the key bits.  Bricks
// with more owned atoms than threads keep cell order.  All threads call.
template <typename T>
__device__ __forceinline__ void rank_owned(const CvArgs<T>& a, const Brick& k, int32_t* keys) {
  constexpr int B = BrickBlock<T>::value, NW = B / 64;
  int32_t* hist = keys + B;               // [NW][kRankBins]: counts, then offsets
  int32_t* start = hist + NW * kRankBins;  // [kRankBins]
  const int32_t* sr = start + kRankBins;   // [B][2]: halo slot, sorted position
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  for (int i = t; i < NW * kRankBins; i += B) hist[i] = 0;
  __syncthreads();
  if (k.O > B) {
    for (int32_t o = t; o < k.O; o += B)
      a.order[k.ob + o] = make_int4(o, a.bi.owned_slot[k.ob + o], a.bi.owned_rank[k.ob + o], 0);
    return;
  }
  const bool act = t < k.O;
  const int key = act ? min(keys[t], kRankBins - 1) : 0;
  if (act) atomicAdd(&hist[w * kRankBins + key], 1);
  __syncthreads();
  if (t < kRankBins) {
    int32_t run = 0;
    for (int v = 0; v < NW; v++) {
      const int32_t c = hist[v * kRankBins + t];
      hist[v * kRankBins + t] = run;
      run += c;
    }
    start[t] = run;  // bucket total for now
  }
  __syncthreads();
  if (t == 0) {
    int32_t run = 0;
    for (int v = kRankBins - 1; v >= 0; v--) {
      const int32_t c = start[v];
      start[v] = run;
      run += c;
    }
  }
  __syncthreads();
  uint64_t same = __ballot(act);
  for (int b = 0; b < 7; b++) {
    const bool bit = (key >> b) & 1;
    const uint64_t m = __ballot(act && bit);
    same &= bit ? m : ~m;
  }
  const int below = __popcll(same & ((1ull << lane) - 1ull));
  if (act)
    a.order[k.ob + start[key] + hist[w * kRankBins + key] + below] = make_int4(t, sr[2 * t], sr[2 * t + 1], 0);
}


// With two lanes per atom, the lanes even out the in-cutoff rows they write:
// the lane with more entries hands its newest ones (still in its shift
// register) to the other, which appends them, so the two parts differ by at
// most one entry (up to 8 move).  The lanes of a wave then walk rows of more
// equal length in passes 2-4 (the parts of one atom are filtered from
// interleaved halves of its list, which split the pairs inside r_c unevenly).
// Both lanes of the pair call this.
__device__ __forceinline__ uint32_t slot_at(const uint4& b, int p) {
  const uint32_t w = p < 2 ? b.x : (p < 4 ? b.y : (p < 6 ? b.z : b.w));
  return (w >> ((p & 1) * 16)) & 0xffffu;
}

__device__ __forceinline__ void balance_pair(SlotWriter& wr) {
  const int32_t mine = wr.n;
  const int32_t other = quad_xor<kQuadXor1>(mine);
  uint4 ob;
  ob.x = (uint32_t)quad_xor<kQuadXor1>((int32_t)wr.buf.x);
  ob.y = (uint32_t)quad_xor<kQuadXor1>((int32_t)wr.buf.y);
  ob.z = (uint32_t)quad_xor<kQuadXor1>((int32_t)wr.buf.z);
  ob.w = (uint32_t)quad_xor<kQuadXor1>((int32_t)wr.buf.w);
  const int32_t give = min(mine > other + 1 ? (mine - other) >> 1 : 0, 8);
  const int32_t take = min(other > mine + 1 ? (other - mine) >> 1 : 0, 8);
  for (int32_t e = 8 - take; e < 8; e++) wr.push((int32_t)slot_at(ob, e));
  if (give == 0) {
    wr.flush();
    return;
  }
  // drop the newest `give`: the partial chunk, if it is still the current one,
  // is written with the kept entries only
  const int32_t keep = mine - give;
  const int32_t r = keep & 7;
  if (r != 0 && (keep >> 3) == (mine >> 3)) {
    uint4 b = wr.buf;
    for (int k = mine & 7; k < 8; k++) {  // the chunk's entries down to the front
      b.x = __builtin_amdgcn_alignbit(b.y, b.x, 16);
      b.y = __builtin_amdgcn_alignbit(b.z, b.y, 16);
      b.z = __builtin_amdgcn_alignbit(b.w, b.z, 16);
      b.w = b.w >> 16;
    }
    uint32_t w[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
    for (int q = 0; q < 8; q++)
      if (q >= r) w[q >> 1] &= (q & 1) ? 0x0000ffffu : 0xffff0000u;
    wr.dst[(keep >> 3) * wr.ps] = make_uint4(w[0], w[1], w[2], w[3]);
  }
  wr.n = keep;
}
// --------------------------------------------------------------------------
// Pass 1
// --------------------------------------------------------------------------
template <typename T, bool CN, bool Q6, bool ALL, bool WRAP>
__device__ __forceinline__ double pass1_atoms(const CvArgs<T>& a, const Brick& k, const vec4_t<T>* lp,
                                              int32_t* keys) {
  double cn_part = 0.0;
  GM_FOR_OWNED(a, k) {
    const int32_t si = a.bi.owned_slot[k.ob + o];
    const int32_t ri = a.bi.owned_rank[k.ob + o];
    const vec4_t<T> pi = fetch_pos<ALL>(a, k, lp, si);
    const int32_t c = min(a.cnt[k.ob + o], a.kmax);
    const int32_t cp = c > part ? ((c - part - 1) >> TSH) + 1 : 0;
    // Phase 1: distance filter over the neighbour sub-row, writing this
    // step's in-cutoff slots (cheap, so divergence costs little).
    uint16_t* crow = a.cut + row_first(a.bg, k.ob, o, part);
    const uint16_t* nrow = a.nbr + row_first(a.bg, k.ob, o, part);
    const int32_t ps = piece_stride(a.bg, k.O);
    // The coordination terms are summed here, on the in-cutoff pairs as they
    // are found: 1/(1 + u^3) with u = (r/r0)^2 needs r^2 only, and so does
    // its gradient, which does not depend on the bias and is kept for the
    // force pass: sum_j -6/r0^2 u^2/(1 + u^3)^2 (x_j - x_i).
    // The in-cutoff rows (and the ranking below) serve the q6 passes 2-4
    // only; the coordination CV alone keeps just their lengths.
    SlotWriter wr;
    wr.init(crow, ps);
    int32_t ncut = 0;
    T cnsum = T(0), gx = T(0), gy = T(0), gz = T(0);
    const T gscale = T(-6) * a.cn_r0inv2;
    for_slots<true>(nrow, cp, ps, first_chunk(nrow, cp), [&](int32_t s) {
      const vec4_t<T> pj = fetch_pos<ALL>(a, k, lp, s);
      T dx, dy, dz;
      const T r2 = pair_vec<WRAP>(pi, pj, a, dx, dy, dz);
      if (r2 < a.rc2) {
        if (Q6)
          wr.push(s);
        else
          ncut++;
        if (CN) {
          const T u = r2 * a.cn_r0inv2;
          const T f = g_rcp(T(1) + u * u * u);
          cnsum += f;
          const T w = u * f;
          const T swp = gscale * w * w;
          gx += swp * dx;
          gy += swp * dy;
          gz += swp * dz;
        }
      }
    });
    if (Q6) {
      if (TPA == 2)
        balance_pair(wr);
      else
        wr.flush();
    }
    const int32_t nc = Q6 ? wr.n : ncut;
    a.ccnt[(int64_t)(k.ob + o) * TPA + part] = nc;
    int32_t longest = nc;
    if (TPA >= 2) longest = max(longest, quad_xor<kQuadXor1>(longest));
    if (TPA >= 4) longest = max(longest, quad_xor<kQuadXor2>(longest));
    if (Q6 && part == 0 && o < BrickBlock<T>::value) {
      keys[o] = longest;
      int32_t* sr = keys + BrickBlock<T>::value * (1 + kRankBins / 64) + kRankBins;
      sr[2 * o] = si;
      sr[2 * o + 1] = ri;
    }
    // Phase 2: the weighted harmonics over the in-cutoff slots only (the
    // thread reads back its own sub-row).
    T Q[13];
#pragma unroll
    for (int m = 0; m < 13; m++) Q[m] = T(0);
    T fsum = T(0);
    if (Q6)
      for_slots<true>(crow, nc, ps, first_chunk(crow, nc), [&](int32_t s) {
        const vec4_t<T> pj = fetch_pos<ALL>(a, k, lp, s);
        T dx, dy, dz;
        const T r2 = pair_vec<WRAP>(pi, pj, a, dx, dy, dz);
        const T rinv = g_rsqrt(r2);
        const T r = r2 * rinv;
        T df;
        const T f = taper_w(r, a, df);
        accumulate_y(a.yc, dx * rinv, dy * rinv, dz * rinv, f, Q);
        fsum += f;
      });
    if (Q6) {
#pragma unroll
      for (int m = 0; m < 13; m++) Q[m] = group_sum(Q[m], TPA);
      fsum = group_sum(fsum, TPA);
    }
    if (CN) {
      cnsum = group_sum(cnsum, TPA);
      gx = group_sum(gx, TPA);
      gy = group_sum(gy, TPA);
      gz = group_sum(gz, TPA);
    }
    if (part == 0) {
      if (Q6) {
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
        store_row16(a.qrow + (int64_t)ri * 16, rowv);
      }
      if (CN) {
        a.cn_atom[ri] = cnsum;
        vec4_t<T> gv;
        gv.x = gx;
        gv.y = gy;
        gv.z = gz;
        gv.w = T(0);
        reinterpret_cast<vec4_t<T>*>(a.cn_grad)[ri] = gv;
        cn_part += (double)cnsum;
      }
    }
  }
  return cn_part;
}

template <typename T, bool CN, bool Q6>
__device__ __forceinline__ void pass1_body(const CvArgs<T>& a, int64_t brick, int32_t blk, int32_t nblk) {
  extern __shared__ __align__(16) unsigned char smem[];
  vec4_t<T>* lp = reinterpret_cast<vec4_t<T>*>(smem);
  __shared__ double red[BrickBlock<T>::value / 64];
  const Brick k = brick_begin(a, brick);
  stage_pos(a, k, lp);
  __syncthreads();
  int32_t* keys = reinterpret_cast<int32_t*>(lp + a.bg.cap);
  const double cn_part = brick_variant(a, k, [&](auto all, auto wrap) {
    return pass1_atoms<T, CN, Q6, decltype(all)::value, decltype(wrap)::value>(a, k, lp, keys);
  });
  if (CN) {
    const double b = block_sum(cn_part, red);
    if (threadIdx.x == 0) (Q6 ? a.part_b : a.part_a)[blk] = b;
  }
  if (Q6) rank_owned(a, k, keys);
}

// --------------------------------------------------------------------------
// Pass 2
// --------------------------------------------------------------------------
template <typename T, bool ALL, bool WRAP>
__device__ __forceinline__ double pass2_atoms(const CvArgs<T>& a, const Brick& k, const vec4_t<T>* lr,
                                              const AtomHead& h0) {
  double c_part = 0.0;
  GM_FOR_RANKED(a, k, h0) {
    vec4_t<T> pi;
    T qi[16];
    fetch_rec<ALL>(a, k, lr, a.qrow, si, pi, qi);
    T nbond = T(0);
    walk_records<ALL>(a, k, lr, a.qrow, a.cut + row_first(a.bg, k.ob, o, part), nc, piece_stride(a.bg, k.O), h.c0, [&](const vec4_t<T>& pj, const T* qj) {
      T dx, dy, dz;
      const T r2 = pair_vec<WRAP>(pi, pj, a, dx, dy, dz);
      const T r = r2 * g_rsqrt(r2);  // the same r as passes 3 and 4
      T df;
      const T f = taper_w(r, a, df);
      T d = T(0);
#pragma unroll
      for (int m = 0; m < 13; m++) d += qi[m] * qj[m];
      nbond += f * logistic((d - a.bond_d0) * a.inv_bond_w);
    });
    nbond = group_sum(nbond, TPA);
    if (part == 0) {
      const T cc = logistic((nbond - a.count_n0) * a.inv_count_w);
      const T dc = cc * (T(1) - cc) * a.inv_count_w;
      a.qrow[(int64_t)ri * 16 + 14] = dc;
      a.nb[ri] = nbond;
      c_part += (double)cc;
    }
  }
  return c_part;
}

template <typename T, bool CN>
__device__ __forceinline__ void pass2_body(const CvArgs<T>& a, int64_t brick, int32_t blk, int32_t nblk) {
  extern __shared__ __align__(16) unsigned char smem[];
  vec4_t<T>* lr = reinterpret_cast<vec4_t<T>*>(smem);
  __shared__ double red[BrickBlock<T>::value / 64];
  const Brick k = brick_begin(a, brick);
  AtomHead h0 = head_begin(a, k);
  stage_rows(a, k, a.qrow, lr);
  head_end(a, k, h0);
  __syncthreads();
  const double c_part = brick_variant(a, k, [&](auto all, auto wrap) {
    return pass2_atoms<T, decltype(all)::value, decltype(wrap)::value>(a, k, lr, h0);
  });
  const double b = block_sum(c_part, red);
  if (threadIdx.x == 0) a.part_a[blk] = b;
}

// --------------------------------------------------------------------------
// Pass 3
// --------------------------------------------------------------------------
template <typename T, bool ALL, bool WRAP>
__device__ __forceinline__ void pass3_atoms(const CvArgs<T>& a, const Brick& k, const vec4_t<T>* lr,
                                            const AtomHead& h0) {
  GM_FOR_RANKED(a, k, h0) {
    vec4_t<T> pi;
    T qi[16];
    fetch_rec<ALL>(a, k, lr, a.qrow, si, pi, qi);
    const T dci = qi[14];
    T hs[13];
#pragma unroll
    for (int m = 0; m < 13; m++) hs[m] = T(0);
    T rx = T(0), ry = T(0), rz = T(0);
    walk_records<ALL>(a, k, lr, a.qrow, a.cut + row_first(a.bg, k.ob, o, part), nc, piece_stride(a.bg, k.O), h.c0, [&](const vec4_t<T>& pj, const T* qj) {
      T dx, dy, dz;
      const T r2 = pair_vec<WRAP>(pi, pj, a, dx, dy, dz);
      const T rinv = g_rsqrt(r2);
      const T r = r2 * rinv;
      T df;
      const T f = taper_w(r, a, df);
      T d = T(0);
#pragma unroll
      for (int m = 0; m < 13; m++) d += qi[m] * qj[m];
      const T b = logistic((d - a.bond_d0) * a.inv_bond_w);
      const T cs = dci + qj[14];
      const T coef = f * b * (T(1) - b) * a.inv_bond_w * cs;
#pragma unroll
      for (int m = 0; m < 13; m++) hs[m] += coef * qj[m];
      // df = 0 below the taper shell: the radial term adds zero there
      const T rad = cs * b * df * rinv;
      rx += rad * dx;
      ry += rad * dy;
      rz += rad * dz;
    });
#pragma unroll
    for (int m = 0; m < 13; m++) hs[m] = group_sum(hs[m], TPA);
    rx = group_sum(rx, TPA);
    ry = group_sum(ry, TPA);
    rz = group_sum(rz, TPA);
    if (part == 0) {
      T proj = T(0);
#pragma unroll
      for (int m = 0; m < 13; m++) proj += qi[m] * hs[m];
      const T inv = qi[13] >= T(1e-12) ? T(1) / qi[13] : T(0);
      T g[16];
#pragma unroll
      for (int m = 0; m < 13; m++) g[m] = (hs[m] - proj * qi[m]) * inv;
      // the taper radial sum rides in the row's last three lanes, which pass 4
      // reads with the atom's own staged record
      g[13] = rx;
      g[14] = ry;
      g[15] = rz;
      store_row16(a.grow + (int64_t)ri * 16, g);
    }
  }
}

template <typename T>
__device__ __forceinline__ void pass3_body(const CvArgs<T>& a, int64_t brick, int32_t blk, int32_t nblk) {
  extern __shared__ __align__(16) unsigned char smem[];
  vec4_t<T>* lr = reinterpret_cast<vec4_t<T>*>(smem);
  const Brick k = brick_begin(a, brick);
  AtomHead h0 = head_begin(a, k);
  stage_rows(a, k, a.qrow, lr);
  head_end(a, k, h0);
  __syncthreads();
  brick_variant(a, k, [&](auto all, auto wrap) {
    pass3_atoms<T, decltype(all)::value, decltype(wrap)::value>(a, k, lr, h0);
  });
}

// --------------------------------------------------------------------------
// Pass 4: chain rule onto positions (u(r) = f(r) v(r_hat) is even in r, so
// both ends of a pair reuse one Jacobian with g_i + g_j).
// --------------------------------------------------------------------------
template <typename T, bool CN, bool ALL, bool WRAP>
__device__ __forceinline__ void pass4_atoms(const CvArgs<T>& a, const Brick& k, const vec4_t<T>* lr,
                                            const AtomHead& h0) {
  const T seed_q = a.seed ? (T)a.seed[a.dims - 1] : T(1);
  const T seed_cn = (CN && a.seed) ? (T)(a.seed[0] * 2.0 * a.inv_n) : T(0);
  GM_FOR_RANKED(a, k, h0) {
    vec4_t<T> pi;
    T gi[16];
    fetch_rec<ALL>(a, k, lr, a.grow, si, pi, gi);
    T ax = T(0), ay = T(0), az = T(0);
    walk_records<ALL>(a, k, lr, a.grow, a.cut + row_first(a.bg, k.ob, o, part), nc, piece_stride(a.bg, k.O), h.c0, [&](const vec4_t<T>& pj, const T* gj) {
      T dx, dy, dz;
      const T r2 = pair_vec<WRAP>(pi, pj, a, dx, dy, dz);
      const T rinv = g_rsqrt(r2);
      const T r = r2 * rinv;
      const T ux = dx * rinv, uy = dy * rinv, uz = dz * rinv;
      T df;
      const T f = taper_w(r, a, df);
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
      const T dS = df * S;  // zero below the taper shell
      px += dS * ux;
      py += dS * uy;
      pz += dS * uz;
      ax += px;
      ay += py;
      az += pz;
    });
    ax = group_sum(ax, TPA);
    ay = group_sum(ay, TPA);
    az = group_sum(az, TPA);
    if (part == 0) {
      // the taper radial sum: the last lanes of the atom's own record, read
      // again here rather than held through the walk
      vec4_t<T> po;
      T go[16];
      fetch_rec<ALL>(a, k, lr, a.grow, si, po, go);
      ax += go[13];
      ay += go[14];
      az += go[15];
      // the coordination gradient, kept by the forward pass
      vec4_t<T> cg;
      cg.x = cg.y = cg.z = cg.w = T(0);
      if (CN) cg = reinterpret_cast<const vec4_t<T>*>(a.cn_grad)[ri];
      write_out(a, ri, -(seed_q * ax + seed_cn * cg.x), -(seed_q * ay + seed_cn * cg.y),
                -(seed_q * az + seed_cn * cg.z));
    }
  }
}

template <typename T, bool CN>
__device__ __forceinline__ void pass4_body(const CvArgs<T>& a, int64_t brick, int32_t blk, int32_t nblk) {
  extern __shared__ __align__(16) unsigned char smem[];
  vec4_t<T>* lr = reinterpret_cast<vec4_t<T>*>(smem);
  const Brick k = brick_begin(a, brick);
  AtomHead h0 = head_begin(a, k);
  stage_rows(a, k, a.grow, lr);
  head_end(a, k, h0);
  __syncthreads();
  brick_variant(a, k, [&](auto all, auto wrap) {
    pass4_atoms<T, CN, decltype(all)::value, decltype(wrap)::value>(a, k, lr, h0);
  });
}

// --------------------------------------------------------------------------
// Coordination number alone: the forces are the seed times the gradient that
// pass 1 kept per atom (ds/dx_i = (2/N) sum_j f'(r_ij) (x_i - x_j)/r_ij, both
// orders of each pair), one thread per owned atom of the brick.
// --------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void cn_force_body(const CvArgs<T>& a, int64_t brick, int32_t blk, int32_t nblk) {
  if (brick >= a.bg.nbricks) return;
  const int32_t ob = a.bi.ob[brick], O = a.bi.ob[brick + 1] - ob;
  const T seed = (T)((a.seed ? a.seed[0] : 1.0) * 2.0 * a.inv_n);
  const vec4_t<T>* g = reinterpret_cast<const vec4_t<T>*>(a.cn_grad);
  for (int32_t o = (int32_t)threadIdx.x; o < O; o += (int32_t)blockDim.x) {
    const int32_t ri = a.bi.owned_rank[ob + o];
    const vec4_t<T> v = g[ri];
    write_out(a, ri, -seed * v.x, -seed * v.y, -seed * v.z);
  }
}

// --------------------------------------------------------------------------
// Kernels: one context (its bricks remapped per XCD), or a batch of contexts
// ("walkers") in one launch.  In a batch, workgroup g (after the same XCD
// remap over the whole grid) belongs to the walker w with
// blk_start[w] <= g < blk_start[w+1] and handles that walker's brick
// g - blk_start[w]; every walker keeps its own partial sums, so
// its results are bitwise the same alone and in a batch.
// --------------------------------------------------------------------------
__device__ __forceinline__ int32_t find_walker(const int32_t* __restrict__ blk_start, int32_t W, int64_t g) {
  int32_t lo = 0, hi = W;
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (blk_start[mid] <= g) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int64_t xcd_remap() {
  const int64_t b = blockIdx.x;
  const int64_t per = gridDim.x / kXcd;
  return (b % kXcd) * per + b / kXcd;
}

// Two brick workgroups share a CU (their staged halos fill its LDS): keep the
// register use of the FP32 passes within what 4 waves per SIMD allow.
#define GM_PASS_OCCUPANCY __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2)))

#define GM_PASS_KERNELS(NAME, BODY, TMPL, TARGS)                                                      \
  TMPL __global__ __launch_bounds__(BrickBlock<T>::value) GM_PASS_OCCUPANCY void NAME(CvArgs<T> a) { \
    const int64_t g = logical_brick(a.bg);                                                            \
    BODY TARGS(a, g, (int32_t)g, (int32_t)gridDim.x);                                                 \
  }                                                                                                   \
  TMPL __global__ __launch_bounds__(BrickBlock<T>::value) GM_PASS_OCCUPANCY void NAME##_batch(         \
      const CvArgs<T>* __restrict__ tab,                                                              \
                                                              const int32_t* __restrict__ blk_start,  \
                                                              int32_t W) {                            \
    const int64_t g = xcd_remap();                                                                    \
    const int32_t w = find_walker(blk_start, W, g);                                                   \
    const int32_t local = (int32_t)(g - blk_start[w]);                                                \
    BODY TARGS(tab[w], local, local, blk_start[w + 1] - blk_start[w]);                                \
  }

#define GM_COMMA ,
GM_PASS_KERNELS(k_pass1, pass1_body, template <typename T GM_COMMA bool CN GM_COMMA bool Q6>, <T GM_COMMA CN GM_COMMA Q6>)
GM_PASS_KERNELS(k_pass2, pass2_body, template <typename T GM_COMMA bool CN>, <T GM_COMMA CN>)
GM_PASS_KERNELS(k_pass3, pass3_body, template <typename T>, <T>)
GM_PASS_KERNELS(k_pass4, pass4_body, template <typename T GM_COMMA bool CN>, <T GM_COMMA CN>)
GM_PASS_KERNELS(k_cn_force, cn_force_body, template <typename T>, <T>)

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
// Launchers
// --------------------------------------------------------------------------
template <typename T>
static size_t lds_bytes(const CvArgs<T>& a, bool rows) {
  return (size_t)a.bg.cap * (size_t)slot_bytes<T>(rows) + (rows ? 0 : (size_t)rank_lds_bytes<T>());
}

template <typename T>
hipError_t launch_q6_forward(const CvArgs<T>& a, bool with_cn, hipStream_t st) {
  const unsigned g = (unsigned)a.bg.blocks;
  if (with_cn) {
    k_pass1<T, true, true><<<g, BrickBlock<T>::value, lds_bytes(a, false), st>>>(a);
    k_pass2<T, true><<<g, BrickBlock<T>::value, lds_bytes(a, true), st>>>(a);
    k_finish<T, true, false><<<1, kBlock, 0, st>>>(a);
  } else {
    k_pass1<T, false, true><<<g, BrickBlock<T>::value, lds_bytes(a, false), st>>>(a);
    k_pass2<T, false><<<g, BrickBlock<T>::value, lds_bytes(a, true), st>>>(a);
    k_finish<T, false, false><<<1, kBlock, 0, st>>>(a);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_q6_adjoint(const CvArgs<T>& a, hipStream_t st) {
  k_pass3<T><<<(unsigned)a.bg.blocks, BrickBlock<T>::value, lds_bytes(a, true), st>>>(a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_q6_force(const CvArgs<T>& a, bool with_cn, hipStream_t st) {
  const unsigned g = (unsigned)a.bg.blocks;
  if (with_cn)
    k_pass4<T, true><<<g, BrickBlock<T>::value, lds_bytes(a, true), st>>>(a);
  else
    k_pass4<T, false><<<g, BrickBlock<T>::value, lds_bytes(a, true), st>>>(a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cn_forward(const CvArgs<T>& a, hipStream_t st) {
  k_pass1<T, true, false><<<(unsigned)a.bg.blocks, BrickBlock<T>::value, lds_bytes(a, false), st>>>(a);
  k_finish<T, false, true><<<1, kBlock, 0, st>>>(a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cn_force(const CvArgs<T>& a, hipStream_t st) {
  k_cn_force<T><<<(unsigned)a.bg.blocks, BrickBlock<T>::value, 0, st>>>(a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_atom_values(const CvArgs<T>& a, int what, int cv_kind, double* dst, hipStream_t st) {
  k_atom_values<T><<<(unsigned)((a.n + kBlock - 1) / kBlock), kBlock, 0, st>>>(a, what, cv_kind, dst);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_pass_batch(int pass, bool with_cn, bool fp_rows, const CvArgs<T>* tab, const int32_t* blk_start,
                             int32_t W, int32_t blocks, int32_t cap, hipStream_t st) {
  const size_t lds_pos = (size_t)cap * slot_bytes<T>(false) + (size_t)rank_lds_bytes<T>(),
               lds_rows = (size_t)cap * slot_bytes<T>(true);
  (void)fp_rows;
  const unsigned g = (unsigned)blocks;
  switch (pass) {
    case 1:
      if (with_cn)
        k_pass1_batch<T, true, true><<<g, BrickBlock<T>::value, lds_pos, st>>>(tab, blk_start, W);
      else
        k_pass1_batch<T, false, true><<<g, BrickBlock<T>::value, lds_pos, st>>>(tab, blk_start, W);
      break;
    case 2:
      if (with_cn) {
        k_pass2_batch<T, true><<<g, BrickBlock<T>::value, lds_rows, st>>>(tab, blk_start, W);
        k_finish_batch<T, true, false><<<(unsigned)W, kBlock, 0, st>>>(tab);
      } else {
        k_pass2_batch<T, false><<<g, BrickBlock<T>::value, lds_rows, st>>>(tab, blk_start, W);
        k_finish_batch<T, false, false><<<(unsigned)W, kBlock, 0, st>>>(tab);
      }
      break;
    case 3:
      k_pass3_batch<T><<<g, BrickBlock<T>::value, lds_rows, st>>>(tab, blk_start, W);
      break;
    case 4:
      if (with_cn)
        k_pass4_batch<T, true><<<g, BrickBlock<T>::value, lds_rows, st>>>(tab, blk_start, W);
      else
        k_pass4_batch<T, false><<<g, BrickBlock<T>::value, lds_rows, st>>>(tab, blk_start, W);
      break;
    case 5:  // coordination alone: forward
      k_pass1_batch<T, true, false><<<g, BrickBlock<T>::value, lds_pos, st>>>(tab, blk_start, W);
      k_finish_batch<T, false, true><<<(unsigned)W, kBlock, 0, st>>>(tab);
      break;
    case 6:  // coordination alone: forces
      k_cn_force_batch<T><<<g, BrickBlock<T>::value, 0, st>>>(tab, blk_start, W);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Allow dynamic LDS up to `bytes` for every staging kernel (ignored where the
// runtime needs no opt-in).
template <typename T>
static void allow_lds_t(int bytes) {
  const hipFuncAttribute A = hipFuncAttributeMaxDynamicSharedMemorySize;
  (void)hipFuncSetAttribute((const void*)k_pass1<T, true, true>, A, bytes);
  (void)hipFuncSetAttribute((const void*)k_pass1<T, false, true>, A, bytes);
  (void)hipFuncSetAttribute((const void*)k_pass1<T, true, false>, A, bytes);
  (void)hipFuncSetAttribute((const void*)k_pass2<T, true>, A, bytes);
  (void)hipFuncSetAttribute((const void*)k_pass2<T, false>, A, bytes);
  (void)hipFuncSetAttribute((const void*)k_pass3<T>, A, bytes);
  (void)hipFuncSetAttribute((const void*)k_pass4<T, true>, A, bytes);
  (void)hipFuncSetAttribute((const void*)k_pass4<T, false>, A, bytes);
  (void)hipFuncSetAttribute((const void*)k_cn_force<T>, A, bytes);
  (void)hipFuncSetAttribute((const void*)k_pass1_batch<T, true, true>, A, bytes);
  (void)hipFuncSetAttribute((const void*)k_pass1_batch<T, false, true>, A, bytes);
  (void)hipFuncSetAttribute((const void*)k_pass1_batch<T, true, false>, A, bytes);
  (void)hipFuncSetAttribute((const void*)k_pass2_batch<T, true>, A, bytes);
  (void)hipFuncSetAttribute((const void*)k_pass2_batch<T, false>, A, bytes);
  (void)hipFuncSetAttribute((const void*)k_pass3_batch<T>, A, bytes);
  (void)hipFuncSetAttribute((const void*)k_pass4_batch<T, true>, A, bytes);
  (void)hipFuncSetAttribute((const void*)k_pass4_batch<T, false>, A, bytes);
  (void)hipFuncSetAttribute((const void*)k_cn_force_batch<T>, A, bytes);
}

void allow_cv_lds(int bytes) {
  allow_lds_t<float>(bytes);
  allow_lds_t<double>(bytes);
  (void)hipGetLastError();
}

#define GM_INSTANTIATE(T)                                                                              \
  template hipError_t launch_q6_forward<T>(const CvArgs<T>&, bool, hipStream_t);                        \
  template hipError_t launch_q6_adjoint<T>(const CvArgs<T>&, hipStream_t);                              \
  template hipError_t launch_q6_force<T>(const CvArgs<T>&, bool, hipStream_t);                          \
  template hipError_t launch_cn_forward<T>(const CvArgs<T>&, hipStream_t);                              \
  template hipError_t launch_cn_force<T>(const CvArgs<T>&, hipStream_t);                                \
  template hipError_t launch_atom_values<T>(const CvArgs<T>&, int, int, double*, hipStream_t);             \
  template hipError_t launch_pass_batch<T>(int, bool, bool, const CvArgs<T>*, const int32_t*, int32_t, int32_t, \
                                           int32_t, hipStream_t);

GM_INSTANTIATE(float)
GM_INSTANTIATE(double)

}  // namespace gm
