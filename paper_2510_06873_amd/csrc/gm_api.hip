// C-ABI of libgpumetad: context, argument validation, call-order state and
// the enqueueing of the kernels in gm_kernels.hip.  No C++ exception crosses
// the boundary; every entry point returns a GM_* code.
#include <math.h>
#include <string.h>

#include <atomic>
#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>

#include <cmath>

#include "gm_internal.h"

using namespace gm;

struct gm_ctx {
  gm_params p;
  int64_t n = 0;
  hipStream_t stream = nullptr;
  int dims = 1;
  bool fp64 = false;
  bool has_q6 = false, has_cn = false;
  bool external = false;  // GM_CV_EXTERNAL: hills only
  double r_list = 0.0;
  double box[3] = {0, 0, 0};
  CellGeom geom;
  BrickGeom bg;
  int64_t ncells = 0, ncells_cap = 0;
  int64_t nbricks_cap = 0, halo_cap = 0, blocks_cap = 0;
  int32_t kmax = 0;
  int bias_blocks = 0;

  // cell list (canonical sorted order)
  int32_t *cell = nullptr, *count = nullptr, *start = nullptr, *perm = nullptr;
  int32_t* scan_tmp = nullptr;  // tile sums of the prefix scans
  // bricks
  int32_t *brick_H = nullptr, *brick_O = nullptr, *brick_hb = nullptr, *brick_ob = nullptr, *brick_hp = nullptr;
  int32_t *halo_rank = nullptr, *owned_slot = nullptr, *owned_rank = nullptr, *owned_hcell = nullptr;
  // neighbour rows and the per-step in-cutoff rows (16-bit halo slots)
  uint16_t *nbr = nullptr, *cut = nullptr;
  int32_t *cnt = nullptr, *ccnt = nullptr, *err = nullptr, *stats = nullptr;
  int4* order = nullptr;  // per brick, by rank: (atom, halo slot, sorted position, 0)
  void *pos_s = nullptr, *qrow = nullptr, *grow = nullptr, *nb = nullptr, *cn_atom = nullptr, *cn_grad = nullptr;
  double *part_a = nullptr, *part_b = nullptr, *s_int = nullptr, *V_int = nullptr, *dV_int = nullptr;
  double *centres = nullptr, *heights = nullptr, *bias_part = nullptr;
  int64_t* hill_count = nullptr;
  BuildArgs* build_dev = nullptr;  // this context's rebuild arguments in device memory (batched rebuilds)
  BuildArgs build_host;            // what build_dev holds (compared before re-uploading)
  bool build_dev_ok = false;

  unsigned char* arena = nullptr;  // the fixed-size buffers below, carved from one allocation
  // buffers that grow or go together, one allocation each: the neighbour and
  // in-cutoff rows; the q-hat and adjoint rows; the cell tables (counts,
  // starts, scan tiles); the brick tables and per-workgroup partials
  unsigned char *rows_blk = nullptr, *qg_blk = nullptr, *cells_blk = nullptr, *bricks_blk = nullptr;
  std::unordered_map<void*, size_t> held;  // device allocations of the context and their sizes
  size_t held_bytes = 0;
  bool built = false, fwd = false, bwd = false;
  const float* fwd_pos = nullptr;  // positions of the last forward pass
  int last_status = GM_OK;
  int64_t version = 0;  // bumped whenever the kernel arguments may change
  uint64_t serial = 0;  // unique per context created in this process
  int lds_budget = 0;   // bytes of dynamic LDS for the staged halo
  YCoef<float> ycf;
  YCoef<double> ycd;
};

namespace {

// Device memory comes from one stream-ordered pool per device: an allocation
// or a free is an operation on the stream it names, so creating and destroying
// contexts and batches while other streams run neither waits for the device
// (as hipFree does) nor maps fresh memory each time; the pool keeps up to
// kPoolKeepBytes cached across synchronisations.
constexpr uint64_t kPoolKeepBytes = 4ull << 30;
constexpr int kMaxDevices = 64;
std::mutex g_pool_mu;
hipMemPool_t g_pool[kMaxDevices] = {};

std::mutex g_lds_mu;
int g_lds_max = 0;  // largest LDS staging budget of any context so far (bytes)

hipMemPool_t device_pool() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_pool_mu);
  if (!g_pool[dev]) {
    hipMemPoolProps pp;
    memset(&pp, 0, sizeof(pp));
    pp.allocType = hipMemAllocationTypePinned;
    pp.handleTypes = hipMemHandleTypeNone;
    pp.location.type = hipMemLocationTypeDevice;
    pp.location.id = dev;
    hipMemPool_t pool = nullptr;
    if (hipMemPoolCreate(&pool, &pp) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    uint64_t keep = kPoolKeepBytes;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    g_pool[dev] = pool;
  }
  return g_pool[dev];
}

// Freed blocks are kept by the library, per device, in size classes (four per
// power of two, at least 64 KiB): a free records an event on its stream and
// files the block; an allocation of the same class takes a filed block that
// was freed on its own stream (stream order covers it) or whose event has
// completed, so neither side blocks the host and no stream waits on another.
// (The pool's own free can wait on the host for several milliseconds when the
// pool hands a block out again, tens of milliseconds under load: in a server
// that retires and admits many walkers at once that idled the device.)  At
// most kCacheKeepBytes stay filed; beyond that the oldest go back to the pool,
// on a library stream that first waits for their events.
constexpr size_t kCacheKeepBytes = 16ull << 30;

struct Filed {
  void* p;
  size_t cls;
  hipStream_t st;  // the stream the block was freed on
  hipEvent_t ev;   // recorded there at the free
};

struct BlockCache {
  std::vector<Filed> filed;       // oldest first
  std::vector<hipEvent_t> spare;  // events free for the next free
  size_t filed_bytes = 0;
  hipStream_t trim = nullptr;
};

struct HandedOut {
  size_t cls;
  int dev;
};

std::mutex g_cache_mu;
BlockCache g_cache[kMaxDevices];
std::unordered_map<void*, HandedOut> g_handed;  // every block handed out

size_t size_class(size_t bytes) {
  size_t g = 64 << 10;
  if (bytes > (256u << 10)) {
    const int top = 63 - __builtin_clzll((unsigned long long)bytes);
    g = (size_t)1 << (top - 2);
  }
  return (bytes + g - 1) / g * g;
}

// A filed block of class cls for st, or null: first one freed on st, then one
// freed on another stream whose free event has completed.  A block freed on st
// whose event is still pending comes with a wait for that event on st (a no-op
// on the device in stream order, and correct if st is a new stream that took
// over the handle of a destroyed one); that event is then destroyed rather than
// recorded again, so that no later record can change what the wait refers to.
void* take_filed(BlockCache& bc, size_t cls, hipStream_t st) {
  for (int pass = 0; pass < 2; pass++)
    for (size_t i = 0; i < bc.filed.size(); i++) {
      const Filed& f = bc.filed[i];
      if (f.cls != cls || (pass == 0 && f.st != st)) continue;
      const bool done = hipEventQuery(f.ev) == hipSuccess;
      if (!done) {
        (void)hipGetLastError();  // not ready is not an error here
        if (pass == 1 || hipStreamWaitEvent(st, f.ev, 0) != hipSuccess) continue;
        (void)hipEventDestroy(f.ev);
      } else {
        bc.spare.push_back(f.ev);
      }
      void* q = f.p;
      bc.filed_bytes -= cls;
      bc.filed.erase(bc.filed.begin() + (std::ptrdiff_t)i);
      return q;
    }
  return nullptr;
}

// Allocate in stream order on st: usable by work enqueued on st after this
// call, and by other streams once ordered after that point.
template <typename P>
int dalloc(hipStream_t st, P** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 16;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return GM_ERR_HIP;
  const size_t cls = size_class(bytes);
  {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    if (void* q = take_filed(g_cache[dev], cls, st)) {
      g_handed[q] = {cls, dev};
      *p = reinterpret_cast<P*>(q);
      return GM_OK;
    }
  }
  hipMemPool_t pool = device_pool();
  if (!pool) return GM_ERR_HIP;
  void* q = nullptr;
  if (hipMallocFromPoolAsync(&q, cls, pool, st) != hipSuccess) {
    (void)hipGetLastError();
    return GM_ERR_OOM;
  }
  std::lock_guard<std::mutex> lock(g_cache_mu);
  g_handed[q] = {cls, dev};
  *p = reinterpret_cast<P*>(q);
  return GM_OK;
}

// Free in stream order on st: the block can be handed out again once the work
// already enqueued on st, which must include every use of it, is done.
template <typename P>
void dfree(hipStream_t st, P*& p) {
  if (!p) return;
  void* q = reinterpret_cast<void*>(p);
  p = nullptr;
  std::lock_guard<std::mutex> lock(g_cache_mu);
  auto it = g_handed.find(q);
  if (it == g_handed.end()) {
    (void)hipFreeAsync(q, st);
    return;
  }
  const HandedOut h = it->second;
  g_handed.erase(it);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != h.dev) {  // filed and trimmed on its own device only
    (void)hipGetLastError();
    (void)hipFreeAsync(q, st);
    return;
  }
  BlockCache& bc = g_cache[h.dev];
  hipEvent_t ev = nullptr;
  if (!bc.spare.empty()) {
    ev = bc.spare.back();
    bc.spare.pop_back();
  } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
    ev = nullptr;
  }
  if (!ev || hipEventRecord(ev, st) != hipSuccess) {  // not filed: back to the pool
    (void)hipGetLastError();
    if (ev) bc.spare.push_back(ev);
    (void)hipFreeAsync(q, st);
    return;
  }
  bc.filed.push_back({q, h.cls, st, ev});
  bc.filed_bytes += h.cls;
  while (bc.filed_bytes > kCacheKeepBytes && !bc.filed.empty()) {
    if (!bc.trim && hipStreamCreateWithFlags(&bc.trim, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      bc.trim = nullptr;
      break;
    }
    const Filed f = bc.filed.front();
    bc.filed.erase(bc.filed.begin());
    bc.filed_bytes -= f.cls;
    (void)hipStreamWaitEvent(bc.trim, f.ev, 0);
    (void)hipFreeAsync(f.p, bc.trim);
    (void)hipEventDestroy(f.ev);
  }
}

// The same for a context's own buffers, which it counts (gm_device_bytes).
template <typename P>
int dalloc_c(gm_ctx* c, P** p, size_t bytes) {
  const int rc = dalloc(c->stream, p, bytes);
  if (rc == GM_OK) {
    const size_t b = bytes == 0 ? 16 : bytes;
    c->held[reinterpret_cast<void*>(*p)] = b;
    c->held_bytes += b;
  }
  return rc;
}

template <typename P>
void dfree_c(gm_ctx* c, P*& p) {
  if (p) {
    auto it = c->held.find(reinterpret_cast<void*>(p));
    if (it != c->held.end()) {
      c->held_bytes -= it->second;
      c->held.erase(it);
    }
  }
  dfree(c->stream, p);
}

#define GM_TRY(x)               \
  do {                          \
    int _rc = (x);              \
    if (_rc != GM_OK) return _rc; \
  } while (0)

// Pieces of one allocation, each on a 256-byte boundary: *p of every piece
// points into *base.  zero_pieces: how many leading pieces are cleared (in
// stream order).  Fewer allocations make creating and destroying a context
// cheaper (a stream-ordered free costs tens of microseconds of host time).
struct Piece {
  void** p;
  size_t bytes;
};

int carve(gm_ctx* c, unsigned char** base, const Piece* pieces, int k, int zero_pieces = 0) {
  size_t total = 0, zero_end = 0;
  for (int i = 0; i < k; i++) {
    total += (pieces[i].bytes + 255) / 256 * 256;
    if (i == zero_pieces - 1) zero_end = total;
  }
  GM_TRY(dalloc_c(c, base, total));
  size_t off = 0;
  for (int i = 0; i < k; i++) {
    *pieces[i].p = *base + off;
    off += (pieces[i].bytes + 255) / 256 * 256;
  }
  if (zero_end && hipMemsetAsync(*base, 0, zero_end, c->stream) != hipSuccess) return GM_ERR_HIP;
  return GM_OK;
}

int hip_rc(hipError_t e) { return e == hipSuccess ? GM_OK : GM_ERR_HIP; }

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

double fact(int k) {
  double f = 1.0;
  for (int i = 2; i <= k; i++) f *= i;
  return f;
}

// Real l = 6 harmonics in polynomial form.  With z = cos(theta) and
// P_6(z) = (231 z^6 - 315 z^4 + 105 z^2 - 5)/16, the m-th derivatives are
//   D1 = (1386 z^5 - 1260 z^3 + 210 z)/16     D2 = (6930 z^4 - 3780 z^2 + 210)/16
//   D3 = (27720 z^3 - 7560 z)/16              D4 = (83160 z^2 - 7560)/16
//   D5 = 166320 z/16                          D6 = 166320/16
// and Y_6m = K_m (-1)^m D_m(z) (x + i y)^m with K_m = sqrt(13/(4 pi) (6-m)!/(6+m)!)
// (Condon-Shortley phase).  The real basis scales m > 0 by sqrt(2).
// The deg real roots in (0, 1) of sum_k p[k] t^k (known to be simple and to
// lie there): sign changes on a fine grid, then bisection to full precision.
void unit_roots(const double* p, int deg, double* out) {
  auto val = [&](double t) {
    double v = p[deg];
    for (int k = deg - 1; k >= 0; k--) v = v * t + p[k];
    return v;
  };
  const int grid = 4096;
  int found = 0;
  double a = 0.0, fa = val(0.0);
  for (int i = 1; i <= grid && found < deg; i++) {
    const double b = (double)i / grid, fb = val(b);
    if ((fa < 0.0) != (fb < 0.0)) {
      double lo = a, hi = b, flo = fa;
      for (int it = 0; it < 200 && hi - lo > 0.0; it++) {
        const double mid = 0.5 * (lo + hi), fm = val(mid);
        if (mid <= lo || mid >= hi) break;
        if ((fm < 0.0) == (flo < 0.0)) {
          lo = mid;
          flo = fm;
        } else {
          hi = mid;
        }
      }
      out[found++] = 0.5 * (lo + hi);
    }
    a = b;
    fa = fb;
  }
  for (; found < deg; found++) out[found] = 0.0;  // not reached for these polynomials
}

template <typename T>
void make_ycoef(YCoef<T>& c) {
  const double D0[4] = {-5, 105, -315, 231}, D1[3] = {210, -1260, 1386}, D2[3] = {210, -3780, 6930};
  const double D3[2] = {-7560, 27720}, D4[2] = {-7560, 83160}, D5 = 166320, D6 = 166320;
  double A[7];
  for (int m = 0; m <= 6; m++) {
    double K = sqrt(13.0 / (4.0 * M_PI) * fact(6 - m) / fact(6 + m));
    A[m] = m == 0 ? K : sqrt(2.0) * ((m & 1) ? -K : K);
  }
  for (int k = 0; k < 4; k++) c.e0[k] = (T)(A[0] * D0[k] / 16.0);
  for (int k = 0; k < 3; k++) c.e1[k] = (T)(A[1] * D1[k] / 16.0);
  for (int k = 0; k < 3; k++) c.e2[k] = (T)(A[2] * D2[k] / 16.0);
  for (int k = 0; k < 2; k++) c.e3[k] = (T)(A[3] * D3[k] / 16.0);
  for (int k = 0; k < 2; k++) c.e4[k] = (T)(A[4] * D4[k] / 16.0);
  c.e5 = (T)(A[5] * D5 / 16.0);
  c.e6 = (T)(A[6] * D6 / 16.0);
  for (int m = 0; m < 6; m++) c.rat[m] = (T)(A[m] / A[m + 1]);
  // Product form: every d^m P_6/dz^m has its 6-m zeros real and inside
  // (-1, 1) (Rolle), so its even/odd part has real roots t = z^2 in (0, 1).
  const double* P[5] = {D0, D1, D2, D3, D4};
  const int deg[5] = {3, 2, 2, 1, 1};
  int at = 0;
  for (int m = 0; m < 5; m++) {
    c.lead[m] = (T)(A[m] * P[m][deg[m]] / 16.0);
    double roots[3];
    unit_roots(P[m], deg[m], roots);
    for (int k = 0; k < deg[m]; k++) c.t[at++] = (T)roots[k];
  }
}

int validate(const gm_params* p, int64_t n) {
  if (!p || p->cv_kind < GM_CV_COORD || p->cv_kind > GM_CV_EXTERNAL) return GM_ERR_INVALID_ARG;
  if (p->precision != GM_FP32 && p->precision != GM_FP64) return GM_ERR_INVALID_ARG;
  for (int d = 0; d < 2; d++)
    if (!(p->period[d] >= 0.0) || !isfinite(p->period[d])) return GM_ERR_INVALID_ARG;
  if (p->cv_kind == GM_CV_EXTERNAL) {
    if (n < 0 || (p->dims != 1 && p->dims != 2)) return GM_ERR_INVALID_ARG;
    for (int d = 0; d < p->dims; d++)
      if (!(p->sigma[d] > 0.0)) return GM_ERR_INVALID_ARG;
    if (!(p->w0 >= 0.0) || !(p->gamma == 0.0 || p->gamma > 1.0)) return GM_ERR_INVALID_ARG;
    if (p->gamma > 1.0 && !(p->kBT > 0.0)) return GM_ERR_INVALID_ARG;
    return p->hill_capacity < 0 ? GM_ERR_INVALID_ARG : GM_OK;
  }
  if (n < 1 || n > (int64_t)INT32_MAX / 2) return GM_ERR_INVALID_ARG;
  if (!(p->r_c > 0.0) || !(p->skin >= 0.0) || !isfinite(p->r_c + p->skin)) return GM_ERR_INVALID_ARG;
  const bool q6 = p->cv_kind != GM_CV_COORD, cn = p->cv_kind != GM_CV_Q6COUNT;
  if (q6 && (!(p->taper > 0.0) || p->taper > p->r_c || !(p->bond_w > 0.0) || !(p->count_w > 0.0)))
    return GM_ERR_INVALID_ARG;
  if (cn && !(p->cn_r0 > 0.0)) return GM_ERR_INVALID_ARG;
  const int dims = p->cv_kind == GM_CV_COORD_Q6 ? 2 : 1;
  for (int d = 0; d < dims; d++)
    if (!(p->sigma[d] > 0.0)) return GM_ERR_INVALID_ARG;
  if (!(p->w0 >= 0.0) || !(p->gamma == 0.0 || p->gamma > 1.0)) return GM_ERR_INVALID_ARG;
  if (p->gamma > 1.0 && !(p->kBT > 0.0)) return GM_ERR_INVALID_ARG;
  if (p->hill_capacity < 0 || p->max_neighbors < 0 || p->max_neighbors > 4096) return GM_ERR_INVALID_ARG;
  for (int a = 0; a < 3; a++)
    if (p->brick[a] < 0 || p->brick[a] > kMaxBrick) return GM_ERR_INVALID_ARG;
  if ((p->brick[0] == 0) != (p->brick[1] == 0) || (p->brick[0] == 0) != (p->brick[2] == 0)) return GM_ERR_INVALID_ARG;
  if (p->lds_kb < 0 || p->lds_kb > 160) return GM_ERR_INVALID_ARG;
  if (p->tpa != 0 && p->tpa != 1 && p->tpa != 2 && p->tpa != 4) return GM_ERR_INVALID_ARG;
  return GM_OK;
}

BrickIndex brick_index(gm_ctx* c) {
  BrickIndex bi;
  bi.hb = c->brick_hb;
  bi.ob = c->brick_ob;
  bi.hp = c->brick_hp;
  bi.halo_rank = c->halo_rank;
  bi.owned_slot = c->owned_slot;
  bi.owned_rank = c->owned_rank;
  bi.owned_hcell = c->owned_hcell;
  return bi;
}

template <typename T>
CvArgs<T> make_args(gm_ctx* c) {
  CvArgs<T> a;
  memset(&a, 0, sizeof(a));
  a.pos_s = reinterpret_cast<const vec4_t<T>*>(c->pos_s);
  a.nbr = c->nbr;
  a.cnt = c->cnt;
  a.cut = c->cut;
  a.ccnt = c->ccnt;
  a.order = c->order;
  a.perm = c->perm;
  a.bg = c->bg;
  a.bi = brick_index(c);
  a.n = c->n;
  a.kmax = c->kmax;
  a.dims = c->dims;
  for (int d = 0; d < 3; d++) {
    const T L = (T)c->box[d];
    a.L[d] = L;
    a.invL[d] = (T)(1.0 / c->box[d]);
    a.Llo[d] = (T)(c->box[d] - (double)L);
  }
  const double rc = c->p.r_c, D = c->p.taper > 0 ? c->p.taper : 1.0;
  a.rc2 = (T)(rc * rc);
  a.taper_lo = (T)(rc - c->p.taper);
  a.pi_over_D = (T)(M_PI / D);
  a.half_pi_over_D = (T)(0.5 * M_PI / D);
  a.bond_d0 = (T)c->p.bond_d0;
  a.inv_bond_w = (T)(c->p.bond_w > 0 ? 1.0 / c->p.bond_w : 0.0);
  a.count_n0 = (T)c->p.count_n0;
  a.inv_count_w = (T)(c->p.count_w > 0 ? 1.0 / c->p.count_w : 0.0);
  a.cn_r0inv2 = (T)(c->p.cn_r0 > 0 ? 1.0 / (c->p.cn_r0 * c->p.cn_r0) : 0.0);
  a.inv_n = 1.0 / (double)c->n;
  if constexpr (sizeof(T) == 4)
    a.yc = c->ycf;
  else
    a.yc = c->ycd;
  a.qrow = reinterpret_cast<T*>(c->qrow);
  a.grow = reinterpret_cast<T*>(c->grow);
  a.nb = reinterpret_cast<T*>(c->nb);
  a.cn_atom = reinterpret_cast<T*>(c->cn_atom);
  a.cn_grad = reinterpret_cast<T*>(c->cn_grad);
  a.part_a = c->part_a;
  a.part_b = c->part_b;
  a.s_int = c->s_int;
  a.err = c->err;
  return a;
}

// Brick size and threads per atom: among the bricks whose expected halo (atoms
// of the (b+2)^3 cells around them, 5% margin) fits the LDS staging budget,
// the one that keeps the most lanes of a 256-thread workgroup busy
// (owned atoms x threads per atom, at most 92% of 256 so that fluctuations
// rarely need a second pass), discounted by the halo re-load ratio.
void choose_bricks(gm_ctx* c, const int32_t nc[3]) {
  const int rec = c->fp64 ? slot_bytes<double>(c->has_q6) : slot_bytes<float>(c->has_q6);
  // pass 1 stages positions only and adds the rank keys; with q6 rows the
  // row staging of passes 2-4 is the larger user
  const int rank = c->fp64 ? rank_lds_bytes<double>() : rank_lds_bytes<float>();
  const int cap = c->has_q6 ? c->lds_budget / rec : (c->lds_budget - rank) / rec;
  const int blk = c->fp64 ? BrickBlock<double>::value : BrickBlock<float>::value;
  const double rho = (double)c->n / ((double)nc[0] * nc[1] * nc[2]);
  int best[3] = {1, 1, 1}, best_tpa = 1;
  double best_score = -1.0;
  const bool fixed = c->p.brick[0] > 0;
  for (int bx = 1; bx <= kMaxBrick && bx <= nc[0]; bx++)
    for (int by = 1; by <= kMaxBrick && by <= nc[1]; by++)
      for (int bz = 1; bz <= kMaxBrick && bz <= nc[2]; bz++) {
        if (fixed && (bx != (c->p.brick[0] < nc[0] ? c->p.brick[0] : nc[0]) ||
                      by != (c->p.brick[1] < nc[1] ? c->p.brick[1] : nc[1]) ||
                      bz != (c->p.brick[2] < nc[2] ? c->p.brick[2] : nc[2])))
          continue;
        const double halo = (double)(bx + 2) * (by + 2) * (bz + 2) * rho;
        const double own = (double)bx * by * bz * rho;
        if (!fixed && halo * 1.05 > cap) continue;
        for (int tpa = 1; tpa <= 4; tpa *= 2) {
          if (c->p.tpa > 0 && tpa != c->p.tpa) continue;
          if (own * tpa > 0.92 * blk && !(fixed && tpa == (c->p.tpa > 0 ? c->p.tpa : 1))) continue;
          const double score = own * tpa * (1.0 - 0.02 * halo / own);
          if (score > best_score) {
            best_score = score;
            best[0] = bx;
            best[1] = by;
            best[2] = bz;
            best_tpa = tpa;
          }
        }
      }
  if (best_score < 0.0 && c->p.tpa > 0) best_tpa = c->p.tpa;  // no brick fits the lanes: 1x1x1
  BrickGeom& g = c->bg;
  for (int a = 0; a < 3; a++) {
    g.nc[a] = nc[a];
    g.b[a] = best[a];
    g.nb[a] = (nc[a] + best[a] - 1) / best[a];
  }
  g.nbricks = g.nb[0] * g.nb[1] * g.nb[2];
  g.cap = cap;
  g.blocks = (g.nbricks + kXcd - 1) / kXcd * kXcd;
  g.tpa = best_tpa;
  g.kpart = ((c->kmax + best_tpa - 1) / best_tpa + 7) / 8 * 8;
  // The neighbour build stages the halo it expects with a margin (slots
  // beyond are read from global memory), so that big-halo systems do not
  // take a CU's LDS for little use; 512 threads when that staging is large
  // (fewer workgroups share a CU), else 256.  A system with few bricks
  // splits each brick's atoms over several workgroups (each stages the
  // whole halo) so that the launch still fills the device, down to about one
  // atom per lane group; the rows are the same for any split.
  const double own = (double)best[0] * best[1] * best[2] * rho;
  const double halo = (double)(best[0] + 2) * (best[1] + 2) * (best[2] + 2) * rho;
  const int bcap = (int)std::ceil(1.25 * halo) + 64;
  g.build_cap = bcap < cap ? bcap : cap;
  g.build_threads = g.build_cap * (int)sizeof(float4) > 32768 ? kBuildMaxThreads : kBlock;
  g.build_split = 1;
  if (g.nbricks < kBuildFillBlocks) {
    int split = (kBuildFillBlocks + g.nbricks - 1) / g.nbricks;
    int most = (int)std::ceil(own / (g.build_threads / kBuildGroup));
    most = most < 1 ? 1 : most;
    split = split < most ? split : most;
    g.build_split = split < kBuildMaxSplit ? split : kBuildMaxSplit;
  }
}

// Upper bound of the total halo slots: each cell is counted once per brick
// whose halo covers it (duplicates included when the halo wraps onto itself).
int64_t halo_bound(const gm_ctx* c) {
  int64_t m = 1;
  for (int a = 0; a < 3; a++) {
    const int n = c->bg.nc[a], b = c->bg.b[a];
    int best = 0;
    int* mult = new int[n]();
    for (int o = 0; o < n; o += b) {
      const int e = b < n - o ? b : n - o;
      for (int p = -1; p <= e; p++) mult[((o + p) % n + n) % n]++;
    }
    for (int i = 0; i < n; i++) best = mult[i] > best ? mult[i] : best;
    delete[] mult;
    m *= best;
  }
  return m * c->n;
}

GatherArgs gather_args(gm_ctx* c, const float* pos4) {
  GatherArgs g;
  g.pos = reinterpret_cast<const float4*>(pos4);
  g.perm = c->perm;
  g.n = c->n;
  g.pos_s = c->pos_s;
  g.err = c->err;
  for (int d = 0; d < 3; d++) g.L[d] = (float)c->geom.L[d];
  return g;
}

BiasArgs make_bias(gm_ctx* c, const double* s, int deposit) {
  BiasArgs b;
  memset(&b, 0, sizeof(b));
  b.s = s;
  b.centres = c->centres;
  b.heights = c->heights;
  b.count = c->hill_count;
  b.capacity = c->p.hill_capacity;
  b.dims = c->dims;
  b.deposit = deposit;
  for (int d = 0; d < c->dims; d++) {
    b.inv2s2[d] = 1.0 / (2.0 * c->p.sigma[d] * c->p.sigma[d]);
    b.invs2[d] = 1.0 / (c->p.sigma[d] * c->p.sigma[d]);
  }
  b.w0 = c->p.w0;
  b.wt_scale = c->p.gamma == 0.0 ? 0.0 : 1.0 / (c->p.kBT * (c->p.gamma - 1.0));
  for (int d = 0; d < 2; d++) b.period[d] = d < c->dims ? c->p.period[d] : 0.0;
  b.part = c->bias_part;
  b.err = c->err;
  return b;
}

void free_all(gm_ctx* c) {
  // every device buffer of a context is carved from one of these
  dfree_c(c, c->arena);
  dfree_c(c, c->rows_blk);
  dfree_c(c, c->qg_blk);
  dfree_c(c, c->cells_blk);
  dfree_c(c, c->bricks_blk);
  dfree_c(c, c->halo_rank);
  c->cell = c->perm = c->owned_slot = c->owned_rank = c->owned_hcell = c->cnt = c->ccnt = nullptr;
  c->err = c->stats = nullptr;
  c->order = nullptr;
  c->pos_s = c->nb = c->cn_atom = c->cn_grad = c->qrow = c->grow = nullptr;
  c->s_int = c->V_int = c->dV_int = c->centres = c->heights = c->bias_part = nullptr;
  c->part_a = c->part_b = nullptr;
  c->hill_count = nullptr;
  c->nbr = c->cut = nullptr;
  c->count = c->start = c->scan_tmp = nullptr;
  c->brick_H = c->brick_O = c->brick_hb = c->brick_ob = c->brick_hp = nullptr;
  c->build_dev = nullptr;
  c->build_dev_ok = false;
}

// The neighbour and in-cutoff rows (tpa sub-rows of kpart entries each).
int alloc_rows(gm_ctx* c) {
  dfree_c(c, c->rows_blk);
  c->nbr = c->cut = nullptr;
  const size_t bytes = (size_t)c->n * (size_t)(c->kmax + 32) * 2;
  const Piece pieces[] = {{(void**)&c->nbr, bytes}, {(void**)&c->cut, bytes}};
  return carve(c, &c->rows_blk, pieces, 2);
}

int status_from_bits(int32_t bits) {
  if (bits & kErrOverflow) return GM_ERR_NEIGHBOR_OVERFLOW;
  if (bits & kErrNonFinite) return GM_ERR_NONFINITE;
  if (bits & kErrCapacity) return GM_ERR_HILL_CAPACITY;
  return GM_OK;
}


}  // namespace

// The per-atom q6 rows (q-hat, adjoint), allocated again after gm_release_rows.
static int ensure_rows(gm_ctx* c) {
  if (!c->has_q6 || c->qg_blk) return GM_OK;
  const size_t bytes = (size_t)c->n * 16 * (c->fp64 ? 8 : 4);
  const Piece pieces[] = {{&c->qrow, bytes}, {&c->grow, bytes}};
  c->version++;
  return carve(c, &c->qg_blk, pieces, 2);
}

template <typename T>
static int cv_forward_t(gm_ctx* c, const float* pos4, double* s_dev) {
  hipStream_t st = c->stream;
  GM_TRY(hip_rc(launch_gather<T>(gather_args(c, pos4), st)));
  CvArgs<T> a = make_args<T>(c);
  a.s_out = s_dev;
  if (c->has_q6) return hip_rc(launch_q6_forward<T>(a, c->has_cn, st));
  return hip_rc(launch_cn_forward<T>(a, st));
}

template <typename T>
static int force_pass(gm_ctx* c, const double* seed, void* out4, int mode) {
  CvArgs<T> a = make_args<T>(c);
  a.seed = seed;
  a.mode = mode;
  a.out4 = out4;
  if (c->has_q6) return hip_rc(launch_q6_force<T>(a, c->has_cn, c->stream));
  return hip_rc(launch_cn_force<T>(a, c->stream));
}

extern "C" {

const char* gm_version(void) { return "gpumetad 0.1 (gfx950)"; }

const char* gm_strerror(int code) {
  switch (code) {
    case GM_OK: return "ok";
    case GM_ERR_INVALID_ARG: return "invalid argument";
    case GM_ERR_OOM: return "device out of memory";
    case GM_ERR_HIP: return "HIP runtime error";
    case GM_ERR_BOX_TOO_SMALL: return "box too small: fewer than 3 cells of width r_c + skin on an axis";
    case GM_ERR_NEIGHBOR_OVERFLOW: return "neighbour list overflow: raise max_neighbors and rebuild";
    case GM_ERR_HILL_CAPACITY: return "hill buffer full";
    case GM_ERR_NONFINITE: return "non-finite position, CV, bias or force";
    case GM_ERR_STATE: return "call out of order";
    case GM_ERR_TOO_LARGE: return "size beyond the fixed scratch of an allocation-free call";
    default: return "unknown error";
  }
}

int gm_create(gm_ctx** out, const gm_params* params, int64_t n_atoms, void* hip_stream) {
  if (!out) return GM_ERR_INVALID_ARG;
  *out = nullptr;
  GM_TRY(validate(params, n_atoms));
  static std::atomic<uint64_t> next_serial{1};
  gm_ctx* c = new (std::nothrow) gm_ctx();
  if (!c) return GM_ERR_OOM;
  c->serial = next_serial.fetch_add(1);
  c->p = *params;
  c->n = n_atoms;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  c->external = params->cv_kind == GM_CV_EXTERNAL;
  c->dims = c->external ? params->dims : (params->cv_kind == GM_CV_COORD_Q6 ? 2 : 1);
  c->fp64 = params->precision == GM_FP64;
  c->has_q6 = !c->external && params->cv_kind != GM_CV_COORD;
  c->has_cn = !c->external && params->cv_kind != GM_CV_Q6COUNT;
  c->r_list = params->r_c + params->skin;
  int32_t km = params->max_neighbors > 0 ? params->max_neighbors : 64;
  c->kmax = (km + 3) / 4 * 4;
  int64_t hb = (params->hill_capacity + kBlock - 1) / kBlock;
  c->bias_blocks = (int)(hb < 1 ? 1 : (hb > 1024 ? 1024 : hb));
  make_ycoef(c->ycf);
  make_ycoef(c->ycd);
  {
    // LDS staging budget: the caller's, else what keeps two workgroups per CU
    // within the device limit (static arrays take the last 2 KiB).
    int dev = 0, lim = 65536;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      lim = 65536;
    (void)hipGetLastError();
    int want = params->lds_kb > 0 ? params->lds_kb * 1024 : 80 * 1024;
    if (want > lim) want = lim;
    c->lds_budget = want - 2048;
    // The kernels' LDS limit is an attribute of the function, shared by every
    // context: keep it at the largest budget any context asked for, so that a
    // context created later with a smaller one does not fail the launches of
    // an earlier one.
    std::lock_guard<std::mutex> lock(g_lds_mu);
    if (c->lds_budget > g_lds_max) g_lds_max = c->lds_budget;
    allow_cv_lds(g_lds_max);
    allow_build_lds(g_lds_max);
  }

  const size_t n = c->external ? 1 : (size_t)n_atoms, T = c->fp64 ? 8 : 4;  // no atom buffers for external CVs
  const size_t cap = (size_t)(params->hill_capacity > 0 ? params->hill_capacity : 1);
  // The buffers whose size is fixed for the life of the context share one
  // allocation; the ones that start at zero come first and are cleared by
  // one memset.
  const Piece pieces[] = {
      {(void**)&c->s_int, 16},       {(void**)&c->V_int, 16},      {(void**)&c->dV_int, 16},
      {(void**)&c->err, 16},         {(void**)&c->stats, 32},      {(void**)&c->hill_count, 16},
      {(void**)&c->nb, n * T},       {(void**)&c->cn_atom, n * T},  // zeroed up to here
      {(void**)&c->cell, n * 4},     {(void**)&c->perm, n * 4},    {(void**)&c->owned_slot, n * 4},
      {(void**)&c->owned_rank, n * 4}, {(void**)&c->owned_hcell, n * 4}, {(void**)&c->cnt, n * 4},
      {(void**)&c->ccnt, n * 4 * 4},  // up to 4 parts per atom
      {(void**)&c->order, n * 16},   {(void**)&c->pos_s, n * 4 * T},
      {(void**)&c->cn_grad, c->has_cn ? n * 4 * T : 16},
      {(void**)&c->centres, cap * c->dims * 8}, {(void**)&c->heights, cap * 8},
      {(void**)&c->bias_part, (size_t)c->bias_blocks * 3 * 8},
      {(void**)&c->build_dev, sizeof(BuildArgs)},
  };
  int rc = carve(c, &c->arena, pieces, (int)(sizeof(pieces) / sizeof(pieces[0])), 8);
  if (rc == GM_OK && !c->external) rc = alloc_rows(c);
  if (rc == GM_OK && c->has_q6) rc = ensure_rows(c);
  if (rc != GM_OK) {
    free_all(c);
    delete c;
    return rc;
  }
  *out = c;
  return GM_OK;
}

int gm_destroy(gm_ctx* c) {
  if (!c) return GM_ERR_INVALID_ARG;
  free_all(c);
  delete c;
  return GM_OK;
}

int gm_set_stream(gm_ctx* c, void* hip_stream) {
  if (!c) return GM_ERR_INVALID_ARG;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  c->version++;
  return GM_OK;
}

// (Re)allocate the brick tables for the current brick geometry.
static int reserve_bricks(gm_ctx* c) {
  const int64_t nbk = c->bg.nbricks, blocks = c->bg.blocks, hbound = halo_bound(c);
  const bool grow_b = nbk > c->nbricks_cap || blocks > c->blocks_cap, grow_h = hbound > c->halo_cap;
  if (grow_b) {
    dfree_c(c, c->bricks_blk);
    const int64_t nb = nbk > c->nbricks_cap ? nbk : c->nbricks_cap;
    const int64_t np = blocks > c->blocks_cap ? blocks : c->blocks_cap;
    c->nbricks_cap = c->blocks_cap = 0;
    const Piece pieces[] = {
        {(void**)&c->brick_H, (size_t)nb * 4},        {(void**)&c->brick_O, (size_t)nb * 4},
        {(void**)&c->brick_hb, (size_t)(nb + 1) * 4}, {(void**)&c->brick_ob, (size_t)(nb + 1) * 4},
        {(void**)&c->brick_hp, (size_t)nb * (kHaloCells + 1) * 4},
        {(void**)&c->part_a, (size_t)np * 8},          {(void**)&c->part_b, (size_t)np * 8},
    };
    GM_TRY(carve(c, &c->bricks_blk, pieces, 7));
    c->nbricks_cap = nb;
    c->blocks_cap = np;
  }
  if (grow_h) {
    dfree_c(c, c->halo_rank);
    c->halo_cap = 0;
    GM_TRY(dalloc_c(c, &c->halo_rank, (size_t)hbound * 4));
    c->halo_cap = hbound;
  }
  return GM_OK;
}

}  // extern "C"

namespace {

// The host half of a rebuild: box checks, cell grid, bricks and the buffers
// they need (allocated in stream order on the context's stream).
int prepare_build(gm_ctx* c, const float* pos4, const double* box) {
  if (c && c->external) return GM_ERR_STATE;
  if (!c || !pos4 || !box || !aligned(pos4, 16)) return GM_ERR_INVALID_ARG;
  int32_t nc[3];
  for (int a = 0; a < 3; a++) {
    if (!(box[a] > 0.0) || !isfinite(box[a])) return GM_ERR_INVALID_ARG;
    double k = floor(box[a] / c->r_list);
    if (k < 3.0) return GM_ERR_BOX_TOO_SMALL;
    if (k > 4096.0) return GM_ERR_INVALID_ARG;
    nc[a] = (int32_t)k;
  }
  const int64_t ncells = (int64_t)nc[0] * nc[1] * nc[2];
  if (ncells > c->ncells_cap) {
    dfree_c(c, c->cells_blk);
    c->ncells_cap = 0;
    const int64_t tiles = (ncells + 1023) / 1024 + 1;  // tile sums of the prefix scans
    const Piece pieces[] = {{(void**)&c->count, (size_t)ncells * 4}, {(void**)&c->start, (size_t)(ncells + 1) * 4},
                            {(void**)&c->scan_tmp, (size_t)tiles * 4}};
    GM_TRY(carve(c, &c->cells_blk, pieces, 3));
    c->ncells_cap = ncells;
  }
  c->ncells = ncells;
  for (int a = 0; a < 3; a++) {
    c->box[a] = box[a];
    c->geom.L[a] = box[a];
    c->geom.inv[a] = (double)nc[a] / box[a];
    c->geom.invL[a] = 1.0 / box[a];
    c->geom.nc[a] = nc[a];
  }
  choose_bricks(c, nc);
  GM_TRY(reserve_bricks(c));
  c->built = c->fwd = c->bwd = false;
  return GM_OK;
}

// The device half, one walker on stream st: canonical cell list (counts,
// scan, scatter, per-cell sort by atom id), brick tables, sorted positions,
// neighbour rows.
int enqueue_build(gm_ctx* c, const float* pos4, hipStream_t st) {
  const int64_t ncells = c->ncells;
  const float4* p4 = reinterpret_cast<const float4*>(pos4);
  // cell counts, list statistics and the out-of-box flag (see the gather)
  GM_TRY(hip_rc(launch_reset_build(c->count, ncells, c->stats, c->err, st)));
  // each atom's slot in its cell goes to owned_slot and the scatter to
  // owned_rank (both rewritten by the brick fill below), then the rank by id
  GM_TRY(hip_rc(launch_cell_ids(p4, c->n, c->geom, c->cell, c->count, c->owned_slot, c->err, st)));
  GM_TRY(hip_rc(launch_scan(c->count, ncells, c->start, nullptr, c->scan_tmp, st)));
  GM_TRY(hip_rc(launch_scatter(c->cell, c->n, c->start, c->owned_slot, c->owned_rank, st)));
  GM_TRY(hip_rc(launch_rank_cells(c->cell, c->start, c->owned_rank, c->n, c->perm, st)));
  // bricks: halo and owned sizes, their prefix sums, the slot tables
  GM_TRY(hip_rc(launch_brick_count(c->start, c->bg, c->brick_H, c->brick_O, st)));
  GM_TRY(hip_rc(launch_scan2(c->brick_H, c->brick_hb, c->brick_O, c->brick_ob, c->bg.nbricks, c->scan_tmp, st)));
  const BrickIndex bi = brick_index(c);
  GM_TRY(hip_rc(launch_brick_fill(c->start, c->bg, bi, c->brick_hp, c->halo_rank, c->owned_slot, c->owned_rank,
                                  c->owned_hcell, c->err, st)));
  const double rl2 = c->r_list * c->r_list;
  if (c->fp64) {
    auto* ps = reinterpret_cast<double4*>(c->pos_s);
    GM_TRY(hip_rc(launch_gather<double>(gather_args(c, pos4), st)));
    GM_TRY(hip_rc(launch_build_nbr<double>(ps, c->geom, c->bg, bi, rl2, c->nbr, c->kmax, c->cnt, c->err, c->stats,
                                           st)));
  } else {
    auto* ps = reinterpret_cast<float4*>(c->pos_s);
    GM_TRY(hip_rc(launch_gather<float>(gather_args(c, pos4), st)));
    GM_TRY(hip_rc(launch_build_nbr<float>(ps, c->geom, c->bg, bi, rl2, c->nbr, c->kmax, c->cnt, c->err, c->stats,
                                          st)));
  }
  return GM_OK;
}

// Every buffer and parameter one rebuild of the context uses (after prepare_build).
BuildArgs build_args(gm_ctx* c, const float* pos4) {
  BuildArgs a;
  memset(&a, 0, sizeof(a));
  a.ga = gather_args(c, pos4);
  a.cg = c->geom;
  a.bg = c->bg;
  a.bi = brick_index(c);
  a.n = c->n;
  a.ncells = c->ncells;
  a.cell = c->cell;
  a.count = c->count;
  a.start = c->start;
  a.slot = c->owned_slot;  // each atom's slot in its cell, rewritten by the brick fill
  a.perm = c->perm;
  a.scat = c->owned_rank;  // the scatter's output, rewritten by the brick fill
  a.stats = c->stats;
  a.err = c->err;
  a.brick_H = c->brick_H;
  a.brick_O = c->brick_O;
  a.brick_hb = c->brick_hb;
  a.brick_ob = c->brick_ob;
  a.brick_hp = c->brick_hp;
  a.halo_rank = c->halo_rank;
  a.owned_slot = c->owned_slot;
  a.owned_rank = c->owned_rank;
  a.owned_hcell = c->owned_hcell;
  a.nbr = c->nbr;
  a.cnt = c->cnt;
  a.kmax = c->kmax;
  a.rl2 = c->r_list * c->r_list;
  return a;
}

}  // namespace

extern "C" {

int gm_build_neighbors(gm_ctx* c, const float* pos4, const double* box) {
  GM_TRY(prepare_build(c, pos4, box));
  GM_TRY(enqueue_build(c, pos4, c->stream));
  c->built = true;
  c->version++;
  return GM_OK;
}

int gm_cv_forward(gm_ctx* c, const float* pos4, double* s_dev) {
  if (!c || !pos4 || !aligned(pos4, 16) || (s_dev && !aligned(s_dev, 8))) return GM_ERR_INVALID_ARG;
  if (!c->built) return GM_ERR_STATE;
  c->fwd = c->bwd = false;
  GM_TRY(ensure_rows(c));
  GM_TRY(c->fp64 ? cv_forward_t<double>(c, pos4, s_dev) : cv_forward_t<float>(c, pos4, s_dev));
  c->fwd = true;
  c->fwd_pos = pos4;
  return GM_OK;
}

int gm_bias_eval(gm_ctx* c, const double* s_dev, double* V_dev, double* dVds_dev) {
  if (!c || !s_dev) return GM_ERR_INVALID_ARG;
  BiasArgs b = make_bias(c, s_dev, 0);
  b.V_out = V_dev;
  b.dV_out = dVds_dev;
  return hip_rc(launch_bias(b, c->bias_blocks, c->stream));
}

int gm_deposit_hill(gm_ctx* c, const double* s_dev) {
  if (!c) return GM_ERR_INVALID_ARG;
  if (!s_dev && !c->fwd) return GM_ERR_STATE;
  BiasArgs b = make_bias(c, s_dev ? s_dev : c->s_int, 1);
  return hip_rc(launch_bias(b, c->bias_blocks, c->stream));
}

int gm_cv_backward(gm_ctx* c, const float* pos4, const double* seed_dev, void* grad4) {
  if (!c || !pos4) return GM_ERR_INVALID_ARG;
  if (!seed_dev && c->dims > 1 && grad4) return GM_ERR_INVALID_ARG;
  const size_t vs = c->fp64 ? 32 : 16;
  if (grad4 && !aligned(grad4, vs)) return GM_ERR_INVALID_ARG;
  if (!c->fwd || pos4 != c->fwd_pos) return GM_ERR_STATE;
  if (c->has_q6) {
    if (c->fp64)
      GM_TRY(hip_rc(launch_q6_adjoint<double>(make_args<double>(c), c->stream)));
    else
      GM_TRY(hip_rc(launch_q6_adjoint<float>(make_args<float>(c), c->stream)));
  }
  c->bwd = true;
  if (grad4) return c->fp64 ? force_pass<double>(c, seed_dev, grad4, 1) : force_pass<float>(c, seed_dev, grad4, 1);
  return GM_OK;
}

int gm_apply_bias_forces(gm_ctx* c, const float* pos4, const double* dVds_dev, void* force4) {
  if (!c || !pos4 || !dVds_dev || !force4) return GM_ERR_INVALID_ARG;
  const size_t vs = c->fp64 ? 32 : 16;
  if (!aligned(force4, vs)) return GM_ERR_INVALID_ARG;
  if (!c->bwd || pos4 != c->fwd_pos) return GM_ERR_STATE;
  return c->fp64 ? force_pass<double>(c, dVds_dev, force4, 0) : force_pass<float>(c, dVds_dev, force4, 0);
}

int gm_hills_get(gm_ctx* c, double* centres, double* heights, int64_t cap, int64_t* k) {
  if (!c || !k) return GM_ERR_INVALID_ARG;
  hipStream_t st = c->stream;
  int64_t K = 0;
  if (hipMemcpyAsync(&K, c->hill_count, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return GM_ERR_HIP;
  *k = K;
  if (centres || heights) {
    if (cap < K) return GM_ERR_INVALID_ARG;
    if (centres && K &&
        hipMemcpyAsync(centres, c->centres, (size_t)K * c->dims * 8, hipMemcpyDeviceToHost, st) != hipSuccess)
      return GM_ERR_HIP;
    if (heights && K && hipMemcpyAsync(heights, c->heights, (size_t)K * 8, hipMemcpyDeviceToHost, st) != hipSuccess)
      return GM_ERR_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return GM_ERR_HIP;
  }
  return GM_OK;
}

int gm_hills_set(gm_ctx* c, const double* centres, const double* heights, int64_t k) {
  if (!c || k < 0 || k > c->p.hill_capacity) return GM_ERR_INVALID_ARG;
  if (k > 0 && (!centres || !heights)) return GM_ERR_INVALID_ARG;
  // in stream order; the wait at the end is for the host buffers to be read
  hipStream_t st = c->stream;
  if (k && hipMemcpyAsync(c->centres, centres, (size_t)k * c->dims * 8, hipMemcpyHostToDevice, st) != hipSuccess)
    return GM_ERR_HIP;
  if (k && hipMemcpyAsync(c->heights, heights, (size_t)k * 8, hipMemcpyHostToDevice, st) != hipSuccess)
    return GM_ERR_HIP;
  if (hipMemcpyAsync(c->hill_count, &k, 8, hipMemcpyHostToDevice, st) != hipSuccess) return GM_ERR_HIP;
  return hipStreamSynchronize(st) == hipSuccess ? GM_OK : GM_ERR_HIP;
}

int gm_hills_set_device(gm_ctx* c, const double* centres_dev, const double* heights_dev, int64_t k) {
  if (!c || k < 0 || k > c->p.hill_capacity) return GM_ERR_INVALID_ARG;
  if (k > 0 && (!centres_dev || !heights_dev || !aligned(centres_dev, 8) || !aligned(heights_dev, 8)))
    return GM_ERR_INVALID_ARG;
  hipStream_t st = c->stream;
  if (k && hipMemcpyAsync(c->centres, centres_dev, (size_t)k * c->dims * 8, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return GM_ERR_HIP;
  if (k && hipMemcpyAsync(c->heights, heights_dev, (size_t)k * 8, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return GM_ERR_HIP;
  // the count goes in through the kernel arguments: nothing waits for the host
  return hip_rc(launch_upload(c->hill_count, &k, 8, st));
}

int gm_status_copy(gm_ctx* c, int32_t* dst) {
  if (!c || !dst || !aligned(dst, 4)) return GM_ERR_INVALID_ARG;
  return hip_rc(hipMemcpyAsync(dst, c->err, 4, hipMemcpyDefault, c->stream));
}

int gm_status_decode(int32_t word) { return status_from_bits(word); }

int gm_status(gm_ctx* c, int sync) {
  if (!c) return GM_ERR_INVALID_ARG;
  if (!sync) return c->last_status;
  int32_t bits = 0;
  if (hipMemcpyAsync(&bits, c->err, 4, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return GM_ERR_HIP;
  if (bits && launch_fill_i32(c->err, 0, 1, c->stream) != hipSuccess) return GM_ERR_HIP;
  c->last_status = status_from_bits(bits);
  return c->last_status;
}

int gm_release_rows(gm_ctx* c) {
  if (!c) return GM_ERR_INVALID_ARG;
  if (c->external) return GM_ERR_STATE;
  if (c->qg_blk) c->version++;
  dfree_c(c, c->qg_blk);
  c->qrow = c->grow = nullptr;
  c->fwd = c->bwd = false;
  return GM_OK;
}

int gm_device_bytes(gm_ctx* c, int64_t* bytes) {
  if (!c || !bytes) return GM_ERR_INVALID_ARG;
  *bytes = (int64_t)c->held_bytes;
  return GM_OK;
}

int gm_neighbor_stats(gm_ctx* c, int32_t* max_count, int64_t* total, int64_t* cutoff_pairs) {
  if (!c) return GM_ERR_INVALID_ARG;
  if (!c->built) return GM_ERR_STATE;
  if (cutoff_pairs) {
    GM_TRY(hip_rc(launch_fill_i32(c->stats + 4, 0, 2, c->stream)));
    if (c->fwd)
      GM_TRY(hip_rc(launch_sum_i32(c->ccnt, c->n * c->bg.tpa, reinterpret_cast<unsigned long long*>(c->stats + 4),
                                   c->stream)));
  }
  int32_t s[8];
  if (hipMemcpyAsync(s, c->stats, 32, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return GM_ERR_HIP;
  if (max_count) *max_count = s[0];
  unsigned long long t;
  if (total) {
    memcpy(&t, &s[2], 8);
    *total = (int64_t)t;
  }
  if (cutoff_pairs) {
    memcpy(&t, &s[4], 8);
    *cutoff_pairs = (int64_t)t;
  }
  return GM_OK;
}

int gm_reserve_neighbors(gm_ctx* c, int32_t max_neighbors) {
  if (c && c->external) return GM_ERR_STATE;
  if (!c || max_neighbors < 1 || max_neighbors > 4096) return GM_ERR_INVALID_ARG;
  c->kmax = (max_neighbors + 3) / 4 * 4;
  c->built = c->fwd = c->bwd = false;
  c->version++;
  return alloc_rows(c);
}

int gm_copy_cell_list(gm_ctx* c, int32_t* perm_dev, int32_t* cell_start_dev, int32_t* ncell) {
  if (c && c->external) return GM_ERR_STATE;
  if (!c || !perm_dev) return GM_ERR_INVALID_ARG;
  if (!c->built) return GM_ERR_STATE;
  if (hipMemcpyAsync(perm_dev, c->perm, (size_t)c->n * 4, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
    return GM_ERR_HIP;
  if (cell_start_dev && hipMemcpyAsync(cell_start_dev, c->start, (size_t)(c->ncells + 1) * 4,
                                       hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
    return GM_ERR_HIP;
  if (ncell)
    for (int a = 0; a < 3; a++) ncell[a] = c->geom.nc[a];
  return GM_OK;
}

int gm_copy_neighbors(gm_ctx* c, int32_t* nbr_dev, int32_t* cnt_dev, int32_t* row_width) {
  if (c && c->external) return GM_ERR_STATE;
  if (!c) return GM_ERR_INVALID_ARG;
  if (!c->built) return GM_ERR_STATE;
  if (row_width) *row_width = c->kmax;
  if (!nbr_dev && !cnt_dev) return GM_OK;
  if (!nbr_dev || !cnt_dev) return GM_ERR_INVALID_ARG;
  return hip_rc(launch_neighbor_ranks(c->nbr, c->cnt, c->bg, brick_index(c), c->kmax, nbr_dev, cnt_dev, c->stream));
}

int gm_atom_values(gm_ctx* c, int what, double* dst_dev) {
  if (c && c->external) return GM_ERR_STATE;
  if (!c || !dst_dev || what < GM_ATOM_Q6 || what > GM_ATOM_CN) return GM_ERR_INVALID_ARG;
  if (!c->fwd) return GM_ERR_STATE;
  if ((what != GM_ATOM_CN && !c->has_q6) || (what == GM_ATOM_CN && !c->has_cn)) return GM_ERR_INVALID_ARG;
  if (c->fp64) return hip_rc(launch_atom_values<double>(make_args<double>(c), what, c->p.cv_kind, dst_dev, c->stream));
  return hip_rc(launch_atom_values<float>(make_args<float>(c), what, c->p.cv_kind, dst_dev, c->stream));
}

}  // extern "C"

// --------------------------------------------------------------------------
// Batches of walkers
// --------------------------------------------------------------------------
struct gm_batch {
  hipStream_t stream = nullptr;
  std::vector<gm_ctx*> walkers;
  std::vector<const float*> pos;
  std::vector<void*> force;
  // A member's entries of the four argument tables, kept while it stays in
  // the batch and recomputed when its context changes (version) or when the
  // entry belongs to another context at the same address (serial).
  struct Entry {
    uint64_t serial = 0;
    int64_t version = -1;
    const float* pos = nullptr;
    void* force = nullptr;
    std::vector<unsigned char> cv, ga, bi, de;
  };
  struct Group {
    int kind = 0;                 // GM_CV_*
    std::vector<int> members;     // indices into walkers
    bool dirty = true;            // members changed since the tables were built
    std::unordered_map<const gm_ctx*, Entry> cache;
    std::vector<unsigned char> h_cv, h_gather, h_bias, h_dep;  // host images of the tables
    std::vector<int32_t> h_blk_cv, h_blk_gather, h_blk_bias;
    void *d_cv = nullptr, *d_gather = nullptr, *d_bias = nullptr, *d_dep = nullptr;
    void *d_blk_cv = nullptr, *d_blk_gather = nullptr, *d_blk_bias = nullptr;
    int32_t blocks_cv = 0, blocks_gather = 0, blocks_bias = 0, cap = 0;
    // capacities of the device tables (kept across membership changes)
    size_t c_cv = 0, c_ga = 0, c_bi = 0, c_de = 0, c_bcv = 0, c_bga = 0, c_bbi = 0;
  };
  std::vector<Group> groups;      // one per CV kind that ever had a member
  bool fp64 = false;
  void* d_vals = nullptr;  // per walker: its s, V and dV/ds buffers (pointers)
  size_t c_vals = 0;
};

namespace {

template <typename T>
void append(std::vector<unsigned char>& v, const T& x) {
  const unsigned char* p = reinterpret_cast<const unsigned char*>(&x);
  v.insert(v.end(), p, p + sizeof(T));
}

// Replace a device table with a host image, in stream order on st (no wait),
// in a buffer of `*cap` bytes kept across calls (grown when too small), so
// that a table whose size does not change keeps its address.
int upload_into(std::vector<unsigned char>& host, void** dev, size_t* cap, hipStream_t st) {
  const size_t need = (host.size() + 3) / 4 * 4;
  if (!*dev || need > *cap) {
    dfree(st, *dev);
    *cap = 0;
    GM_TRY(dalloc(st, dev, need));
    *cap = need;
  }
  return hip_rc(launch_upload(*dev, host.data(), host.size(), st));
}

int upload_into_i32(const std::vector<int32_t>& v, void** dev, size_t* cap, hipStream_t st) {
  std::vector<unsigned char> h(reinterpret_cast<const unsigned char*>(v.data()),
                               reinterpret_cast<const unsigned char*>(v.data()) + v.size() * 4);
  return upload_into(h, dev, cap, st);
}

// Bring the device tables of a group up to date: the entries of members whose
// context changed since the last call are recomputed, and a table is uploaded
// only if its bytes changed (into the same device buffer when it fits).
template <typename T>
int refresh_group(gm_batch* B, gm_batch::Group& g, bool force) {
  const size_t W = g.members.size();
  bool stale = force || g.dirty;
  for (size_t i = 0; !stale && i < W; i++) {
    const int m = g.members[i];
    const gm_ctx* c = B->walkers[m];
    auto it = g.cache.find(c);
    stale = it == g.cache.end() || it->second.serial != c->serial || it->second.version != c->version ||
            it->second.pos != B->pos[m] || it->second.force != B->force[m];
  }
  if (!stale) return GM_OK;
  std::vector<int32_t> bcv{0}, bga{0}, bbi{0};
  std::vector<unsigned char> cv, ga, bi, de;
  g.cap = 0;
  for (size_t i = 0; i < W; i++) {
    const int m = g.members[i];
    gm_ctx* c = B->walkers[m];
    if (!c->built) return GM_ERR_STATE;
    GM_TRY(ensure_rows(c));
    gm_batch::Entry& e = g.cache[c];
    if (force || e.serial != c->serial || e.version != c->version || e.pos != B->pos[m] || e.force != B->force[m]) {
      CvArgs<T> a = make_args<T>(c);
      a.s_out = nullptr;
      a.seed = c->dV_int;
      a.mode = 0;
      a.out4 = B->force[m];
      e.cv.clear();
      append(e.cv, a);
      e.ga.clear();
      append(e.ga, gather_args(c, B->pos[m]));
      BiasArgs ev = make_bias(c, c->s_int, 0);
      ev.V_out = c->V_int;
      ev.dV_out = c->dV_int;
      e.bi.clear();
      append(e.bi, ev);
      e.de.clear();
      append(e.de, make_bias(c, c->s_int, 1));
      e.serial = c->serial;
      e.version = c->version;
      e.pos = B->pos[m];
      e.force = B->force[m];
    }
    cv.insert(cv.end(), e.cv.begin(), e.cv.end());
    ga.insert(ga.end(), e.ga.begin(), e.ga.end());
    bi.insert(bi.end(), e.bi.begin(), e.bi.end());
    de.insert(de.end(), e.de.begin(), e.de.end());
    bcv.push_back(bcv.back() + c->bg.blocks);
    bga.push_back(bga.back() + (int32_t)((c->n + kBlock - 1) / kBlock));
    bbi.push_back(bbi.back() + c->bias_blocks);
    g.cap = c->bg.cap > g.cap ? c->bg.cap : g.cap;
  }
  g.blocks_cv = bcv.back();
  g.blocks_gather = bga.back();
  g.blocks_bias = bbi.back();
  if (force || cv != g.h_cv) GM_TRY(upload_into(cv, &g.d_cv, &g.c_cv, B->stream));
  if (force || ga != g.h_gather) GM_TRY(upload_into(ga, &g.d_gather, &g.c_ga, B->stream));
  if (force || bi != g.h_bias) GM_TRY(upload_into(bi, &g.d_bias, &g.c_bi, B->stream));
  if (force || de != g.h_dep) GM_TRY(upload_into(de, &g.d_dep, &g.c_de, B->stream));
  if (force || bcv != g.h_blk_cv) GM_TRY(upload_into_i32(bcv, &g.d_blk_cv, &g.c_bcv, B->stream));
  if (force || bga != g.h_blk_gather) GM_TRY(upload_into_i32(bga, &g.d_blk_gather, &g.c_bga, B->stream));
  if (force || bbi != g.h_blk_bias) GM_TRY(upload_into_i32(bbi, &g.d_blk_bias, &g.c_bbi, B->stream));
  g.h_blk_cv.swap(bcv);
  g.h_blk_gather.swap(bga);
  g.h_blk_bias.swap(bbi);
  g.h_cv.swap(cv);
  g.h_gather.swap(ga);
  g.h_bias.swap(bi);
  g.h_dep.swap(de);
  g.dirty = false;
  return GM_OK;
}

template <typename T>
int batch_step_t(gm_batch* B) {
  for (auto& g : B->groups) {
    if (g.members.empty()) continue;
    GM_TRY(refresh_group<T>(B, g, false));
    const int32_t W = (int32_t)g.members.size();
    auto* tab = reinterpret_cast<const CvArgs<T>*>(g.d_cv);
    const auto* bcv = static_cast<const int32_t*>(g.d_blk_cv);
    const bool q6 = g.kind != GM_CV_COORD, cn = g.kind != GM_CV_Q6COUNT;
    hipStream_t st = B->stream;
    GM_TRY(hip_rc(launch_gather_batch<T>(reinterpret_cast<const GatherArgs*>(g.d_gather),
                                         static_cast<const int32_t*>(g.d_blk_gather), W, g.blocks_gather, st)));
    if (q6) {
      GM_TRY(hip_rc(launch_pass_batch<T>(1, cn, true, tab, bcv, W, g.blocks_cv, g.cap, st)));
      GM_TRY(hip_rc(launch_pass_batch<T>(2, cn, true, tab, bcv, W, g.blocks_cv, g.cap, st)));
    } else {
      GM_TRY(hip_rc(launch_pass_batch<T>(5, true, false, tab, bcv, W, g.blocks_cv, g.cap, st)));
    }
    GM_TRY(hip_rc(launch_bias_batch(reinterpret_cast<const BiasArgs*>(g.d_bias),
                                    static_cast<const int32_t*>(g.d_blk_bias), W, g.blocks_bias, st)));
    if (q6) {
      GM_TRY(hip_rc(launch_pass_batch<T>(3, cn, true, tab, bcv, W, g.blocks_cv, g.cap, st)));
      GM_TRY(hip_rc(launch_pass_batch<T>(4, cn, true, tab, bcv, W, g.blocks_cv, g.cap, st)));
    } else {
      GM_TRY(hip_rc(launch_pass_batch<T>(6, true, false, tab, bcv, W, g.blocks_cv, g.cap, st)));
    }
    for (int m : g.members) {
      gm_ctx* c = B->walkers[m];
      c->fwd = c->bwd = true;
      c->fwd_pos = B->pos[m];
    }
  }
  return GM_OK;
}

void free_batch(gm_batch* B) {
  dfree(B->stream, B->d_vals);
  for (auto& g : B->groups) {
    dfree(B->stream, g.d_cv);
    dfree(B->stream, g.d_gather);
    dfree(B->stream, g.d_bias);
    dfree(B->stream, g.d_dep);
    dfree(B->stream, g.d_blk_cv);
    dfree(B->stream, g.d_blk_gather);
    dfree(B->stream, g.d_blk_bias);
  }
}

}  // namespace

extern "C" {

// ---- CVs of a few atoms, lattice parameters, free energy --------------------
namespace {
bool box_ok(const double* b) {
  return b && b[0] > 0.0 && b[1] > 0.0 && b[2] > 0.0 && isfinite(b[0]) && isfinite(b[1]) && isfinite(b[2]);
}
bool force_ok(const void* f, int32_t precision) {
  return f && (precision == GM_FP32 || precision == GM_FP64) && aligned(f, precision == GM_FP64 ? 32 : 16);
}
}  // namespace

int gm_torsions(const float* pos4, int64_t n_atoms, const int32_t* quads_dev, int32_t count, const double* box,
                double* phi_dev, void* hip_stream) {
  if (count < 0 || count > kMaxTorsions) return GM_ERR_INVALID_ARG;
  if (count == 0) return GM_OK;
  if (!pos4 || !aligned(pos4, 16) || n_atoms < 1 || !quads_dev || !aligned(quads_dev, 4) || !phi_dev ||
      !aligned(phi_dev, 8) || !box_ok(box))
    return GM_ERR_INVALID_ARG;
  return hip_rc(launch_torsions(reinterpret_cast<const float4*>(pos4), n_atoms, quads_dev, count, box, phi_dev,
                                reinterpret_cast<hipStream_t>(hip_stream)));
}

int gm_torsion_forces(const float* pos4, int64_t n_atoms, const int32_t* quads_dev, int32_t count, const double* box,
                      const double* dVdphi_dev, void* force4, int32_t precision, void* hip_stream) {
  if (count < 0 || count > kMaxTorsions) return GM_ERR_INVALID_ARG;
  if (count == 0) return GM_OK;
  if (!pos4 || !aligned(pos4, 16) || n_atoms < 1 || !quads_dev || !aligned(quads_dev, 4) || !dVdphi_dev ||
      !aligned(dVdphi_dev, 8) || !force_ok(force4, precision) || !box_ok(box))
    return GM_ERR_INVALID_ARG;
  return hip_rc(launch_torsion_forces(reinterpret_cast<const float4*>(pos4), n_atoms, quads_dev, count, box,
                                      dVdphi_dev, force4, precision == GM_FP64,
                                      reinterpret_cast<hipStream_t>(hip_stream)));
}

int gm_nearest_distance(const float* pos4, int64_t n_atoms, int32_t centre, const int32_t* members_dev,
                        int32_t count, const double* box, double* s_dev, int32_t* nearest_dev, void* hip_stream) {
  if (!pos4 || !aligned(pos4, 16) || n_atoms < 1 || centre < 0 || centre >= n_atoms || !members_dev ||
      !aligned(members_dev, 4) || count < 1 || !s_dev || !aligned(s_dev, 8) ||
      (nearest_dev && !aligned(nearest_dev, 4)) || !box_ok(box))
    return GM_ERR_INVALID_ARG;
  return hip_rc(launch_nearest(reinterpret_cast<const float4*>(pos4), n_atoms, centre, members_dev, count, box, s_dev,
                               nearest_dev, nullptr, nullptr, false, reinterpret_cast<hipStream_t>(hip_stream)));
}

int gm_nearest_distance_forces(const float* pos4, int64_t n_atoms, int32_t centre, const int32_t* members_dev,
                               int32_t count, const double* box, const double* dVds_dev, void* force4,
                               int32_t precision, void* hip_stream) {
  if (!pos4 || !aligned(pos4, 16) || n_atoms < 1 || centre < 0 || centre >= n_atoms || !members_dev ||
      !aligned(members_dev, 4) || count < 1 || !dVds_dev || !aligned(dVds_dev, 8) || !force_ok(force4, precision) ||
      !box_ok(box))
    return GM_ERR_INVALID_ARG;
  return hip_rc(launch_nearest(reinterpret_cast<const float4*>(pos4), n_atoms, centre, members_dev, count, box,
                               nullptr, nullptr, dVds_dev, force4, precision == GM_FP64,
                               reinterpret_cast<hipStream_t>(hip_stream)));
}

int gm_lattice_virial(const double* box, const double* dVdL, int32_t dims, double* virial) {
  if (!box || !dVdL || !virial || dims < 1 || dims > 3) return GM_ERR_INVALID_ARG;
  for (int a = 0; a < dims; a++) virial[a] = -box[a] * dVdL[a];
  return GM_OK;
}

int gm_fes_reweight(const double* s_dev, const double* V_dev, int64_t T, int32_t dims, const double* lo,
                    const double* hi, const int32_t* nbins, double kBT, double* F_dev, void* hip_stream) {
  if (!s_dev || !V_dev || !F_dev || !lo || !hi || !nbins || T < 1 || (dims != 1 && dims != 2) || !(kBT > 0.0) ||
      !aligned(s_dev, 8) || !aligned(V_dev, 8) || !aligned(F_dev, 8))
    return GM_ERR_INVALID_ARG;
  int64_t total = 1;
  for (int d = 0; d < dims; d++) {
    if (nbins[d] < 1 || !(hi[d] > lo[d]) || !isfinite(lo[d]) || !isfinite(hi[d])) return GM_ERR_INVALID_ARG;
    total *= nbins[d];
  }
  if (total > kMaxFesBins) return GM_ERR_INVALID_ARG;
  static std::once_flag lds_once;
  std::call_once(lds_once, allow_fes_lds);
  return hip_rc(launch_fes_reweight(s_dev, V_dev, T, dims, lo, hi, nbins, kBT, F_dev,
                                    reinterpret_cast<hipStream_t>(hip_stream)));
}

int gm_fes_reweight_noalloc(const double* s_dev, const double* V_dev, int64_t T, int32_t dims, const double* lo,
                            const double* hi, const int32_t* nbins, double kBT, double* F_dev, void* hip_stream) {
  if (!s_dev || !V_dev || !F_dev || !lo || !hi || !nbins || T < 1 || (dims != 1 && dims != 2) || !(kBT > 0.0) ||
      !aligned(s_dev, 8) || !aligned(V_dev, 8) || !aligned(F_dev, 8))
    return GM_ERR_INVALID_ARG;
  int64_t total = 1;
  for (int d = 0; d < dims; d++) {
    if (nbins[d] < 1 || !(hi[d] > lo[d]) || !isfinite(lo[d]) || !isfinite(hi[d])) return GM_ERR_INVALID_ARG;
    total *= nbins[d];
    if (total > kFesNoAllocMaxBins) return GM_ERR_TOO_LARGE;
  }
  static std::once_flag lds_once;
  std::call_once(lds_once, allow_fes_lds);
  return hip_rc(launch_fes_reweight_noalloc(s_dev, V_dev, T, dims, lo, hi, nbins, kBT, F_dev,
                                            reinterpret_cast<hipStream_t>(hip_stream)));
}

int gm_fes_hills(gm_ctx* c, const double* lo, const double* hi, const int32_t* nbins, double* F_dev) {
  if (!c || !lo || !hi || !nbins || !F_dev || !aligned(F_dev, 8)) return GM_ERR_INVALID_ARG;
  int64_t total = 1;
  for (int d = 0; d < c->dims; d++) {
    if (nbins[d] < 1 || !(hi[d] > lo[d]) || !isfinite(lo[d]) || !isfinite(hi[d])) return GM_ERR_INVALID_ARG;
    total *= nbins[d];
  }
  if (total > kMaxFesBins) return GM_ERR_INVALID_ARG;
  const double scale = c->p.gamma > 1.0 ? c->p.gamma / (c->p.gamma - 1.0) : 1.0;
  return hip_rc(launch_fes_hills(make_bias(c, nullptr, 0), lo, hi, nbins, scale, F_dev, c->stream));
}

}  // extern "C"

namespace {

// Validate a member list (distinct internal-CV contexts of the batch's
// precision, aligned arrays) and make it the batch's: groups by CV kind keep
// their device tables and the cached entries of members that stay; walkers
// are bound to the batch stream; the table of value pointers is re-uploaded.
int set_members(gm_batch* B, gm_ctx* const* walkers, int32_t count, const float* const* pos4, void* const* force4) {
  const size_t vs = B->fp64 ? 32 : 16;
  for (int32_t i = 0; i < count; i++) {
    gm_ctx* c = walkers[i];
    if (!c || c->external || !pos4[i] || !force4[i] || c->fp64 != B->fp64 || !aligned(pos4[i], 16) ||
        !aligned(force4[i], vs))
      return GM_ERR_INVALID_ARG;
    for (int32_t j = 0; j < i; j++)
      if (walkers[j] == c) return GM_ERR_INVALID_ARG;
  }
  B->walkers.assign(walkers, walkers + count);
  B->pos.assign(pos4, pos4 + count);
  B->force.assign(force4, force4 + count);
  for (int kind = GM_CV_COORD; kind <= GM_CV_COORD_Q6; kind++) {
    gm_batch::Group* g = nullptr;
    for (auto& h : B->groups)
      if (h.kind == kind) g = &h;
    std::vector<int> members;
    for (int32_t i = 0; i < count; i++)
      if (walkers[i]->p.cv_kind == kind) members.push_back(i);
    if (!g) {
      if (members.empty()) continue;
      B->groups.emplace_back();
      g = &B->groups.back();
      g->kind = kind;
    }
    g->members.swap(members);
    g->dirty = true;
    // forget the entries of contexts that left (they may be destroyed, and a
    // new context may later take the same address)
    for (auto it = g->cache.begin(); it != g->cache.end();) {
      bool stays = false;
      for (int m : g->members) stays = stays || B->walkers[m] == it->first;
      it = stays ? std::next(it) : g->cache.erase(it);
    }
  }
  for (gm_ctx* c : B->walkers)
    if (c->stream != B->stream) {
      c->stream = B->stream;
      c->version++;
    }
  if (count == 0) return GM_OK;
  std::vector<unsigned char> vals;
  for (gm_ctx* c : B->walkers) {
    append(vals, c->s_int);
    append(vals, c->V_int);
    append(vals, c->dV_int);
  }
  const int rc = upload_into(vals, &B->d_vals, &B->c_vals, B->stream);
  if (rc != GM_OK) {
    // no table of value pointers for these members: leave the batch empty
    B->walkers.clear();
    B->pos.clear();
    B->force.clear();
    for (auto& g : B->groups) {
      g.members.clear();
      g.dirty = true;
    }
  }
  return rc;
}

}  // namespace

extern "C" {

int gm_batch_create(gm_batch** out, gm_ctx* const* walkers, int32_t count, const float* const* pos4,
                    void* const* force4, void* hip_stream) {
  if (!out) return GM_ERR_INVALID_ARG;
  *out = nullptr;
  if (!walkers || !pos4 || !force4 || count < 1 || !walkers[0]) return GM_ERR_INVALID_ARG;
  gm_batch* B = new (std::nothrow) gm_batch();
  if (!B) return GM_ERR_OOM;
  B->stream = reinterpret_cast<hipStream_t>(hip_stream);
  B->fp64 = walkers[0]->fp64;
  const int rc = set_members(B, walkers, count, pos4, force4);
  if (rc != GM_OK) {
    free_batch(B);
    delete B;
    return rc;
  }
  *out = B;
  return GM_OK;
}

int gm_batch_update(gm_batch* B, gm_ctx* const* walkers, int32_t count, const float* const* pos4,
                    void* const* force4) {
  if (!B || count < 0 || (count > 0 && (!walkers || !pos4 || !force4))) return GM_ERR_INVALID_ARG;
  return set_members(B, walkers, count, pos4, force4);
}

int gm_batch_destroy(gm_batch* B) {
  if (!B) return GM_ERR_INVALID_ARG;
  free_batch(B);
  delete B;
  return GM_OK;
}

}  // extern "C"

namespace {

// Rebuild the listed members on stream st: host preparation for each, then
// the batchable ones one launch per stage (kBuildSubsetMax at a time), the
// rest alone.  The walkers' own streams are st meanwhile, so that buffers
// grown here are allocated and released in the order of st.
int batch_build(gm_batch* B, const int32_t* which, int32_t count, const double* boxes, hipStream_t st) {
  const int32_t W = (int32_t)B->walkers.size();
  std::vector<char> seen(W, 0);
  for (int32_t i = 0; i < count; i++) {
    if (which[i] < 0 || which[i] >= W || seen[which[i]]) return GM_ERR_INVALID_ARG;
    seen[which[i]] = 1;
  }
  struct Restore {
    gm_batch* B;
    const int32_t* which;
    int32_t count;
    ~Restore() {
      for (int32_t i = 0; i < count; i++) B->walkers[which[i]]->stream = B->stream;
    }
  } restore{B, which, count};
  for (int32_t i = 0; i < count; i++) B->walkers[which[i]]->stream = st;
  for (int32_t i = 0; i < count; i++) GM_TRY(prepare_build(B->walkers[which[i]], B->pos[which[i]], boxes + 3 * i));
  std::vector<const BuildArgs*> dev;
  std::vector<BuildArgs> host;
  auto flush = [&]() -> int {
    const int rc = hip_rc(launch_build_batch(dev.data(), host.data(), (int32_t)dev.size(), B->fp64, st));
    dev.clear();
    host.clear();
    return rc;
  };
  for (int32_t i = 0; i < count; i++) {
    gm_ctx* c = B->walkers[which[i]];
    const float* pos4 = B->pos[which[i]];
    const BuildArgs a = build_args(c, pos4);
    if (!build_batchable(a)) {
      GM_TRY(enqueue_build(c, pos4, st));
      continue;
    }
    if (!c->build_dev_ok || memcmp(&a, &c->build_host, sizeof(a)) != 0) {
      GM_TRY(hip_rc(launch_upload(c->build_dev, &a, sizeof(a), st)));
      c->build_host = a;
      c->build_dev_ok = true;
    }
    dev.push_back(c->build_dev);
    host.push_back(a);
    if ((int)dev.size() == kBuildSubsetMax) GM_TRY(flush());
  }
  if (!dev.empty()) GM_TRY(flush());
  for (int32_t i = 0; i < count; i++) {
    gm_ctx* c = B->walkers[which[i]];
    c->built = true;
    c->version++;
  }
  return GM_OK;
}

}  // namespace

extern "C" {

int gm_batch_build(gm_batch* B, const double* boxes) {
  if (!B || !boxes) return GM_ERR_INVALID_ARG;
  std::vector<int32_t> all(B->walkers.size());
  for (size_t i = 0; i < all.size(); i++) all[i] = (int32_t)i;
  return batch_build(B, all.data(), (int32_t)all.size(), boxes, B->stream);
}

int gm_batch_build_some(gm_batch* B, const int32_t* which, int32_t count, const double* boxes, void* hip_stream) {
  if (!B || count < 0 || (count > 0 && (!which || !boxes))) return GM_ERR_INVALID_ARG;
  hipStream_t st = hip_stream ? reinterpret_cast<hipStream_t>(hip_stream) : B->stream;
  return batch_build(B, which, count, boxes, st);
}

int gm_batch_step(gm_batch* B) {
  if (!B) return GM_ERR_INVALID_ARG;
  for (gm_ctx* c : B->walkers)
    if (!c->built) return GM_ERR_STATE;
  return B->fp64 ? batch_step_t<double>(B) : batch_step_t<float>(B);
}

int gm_batch_deposit(gm_batch* B) {
  if (!B) return GM_ERR_INVALID_ARG;
  for (auto& g : B->groups) {
    if (g.members.empty()) continue;
    GM_TRY(B->fp64 ? refresh_group<double>(B, g, false) : refresh_group<float>(B, g, false));
    GM_TRY(hip_rc(launch_bias_batch(reinterpret_cast<const BiasArgs*>(g.d_dep), static_cast<const int32_t*>(g.d_blk_bias),
                                    (int32_t)g.members.size(), g.blocks_bias, B->stream)));
  }
  return GM_OK;
}

int gm_batch_deposit_some(gm_batch* B, const int32_t* which, int32_t count) {
  if (!B || count < 0 || (count > 0 && !which)) return GM_ERR_INVALID_ARG;
  const int32_t W = (int32_t)B->walkers.size();
  std::vector<char> seen(W, 0);
  for (int32_t i = 0; i < count; i++) {
    if (which[i] < 0 || which[i] >= W || seen[which[i]]) return GM_ERR_INVALID_ARG;
    if (!B->walkers[which[i]]->fwd) return GM_ERR_STATE;
    seen[which[i]] = 1;
  }
  for (auto& g : B->groups) {
    bool any = false;
    for (int m : g.members) any = any || seen[m];
    if (any) GM_TRY(B->fp64 ? refresh_group<double>(B, g, false) : refresh_group<float>(B, g, false));
  }
  BiasSubset s;
  s.k = 0;
  s.blk[0] = 0;
  for (int32_t i = 0; i < count; i++) {
    const int m = which[i];
    const gm_batch::Group* gp = nullptr;
    int pos = -1;
    for (const auto& g : B->groups)
      for (size_t j = 0; j < g.members.size() && pos < 0; j++)
        if (g.members[j] == m) {
          gp = &g;
          pos = (int)j;
        }
    if (!gp) return GM_ERR_INVALID_ARG;
    s.tab[s.k] = reinterpret_cast<const BiasArgs*>(gp->d_dep) + pos;
    s.blk[s.k + 1] = s.blk[s.k] + B->walkers[m]->bias_blocks;
    if (++s.k == kSubsetMax || i == count - 1) {
      GM_TRY(hip_rc(launch_bias_subset(s, B->stream)));
      s.k = 0;
    }
  }
  return GM_OK;
}

int gm_batch_values(gm_batch* B, double* s_dev, double* V_dev, double* dVds_dev) {
  if (!B) return GM_ERR_INVALID_ARG;
  if ((s_dev && !aligned(s_dev, 8)) || (V_dev && !aligned(V_dev, 8)) || (dVds_dev && !aligned(dVds_dev, 8)))
    return GM_ERR_INVALID_ARG;
  if ((!s_dev && !V_dev && !dVds_dev) || B->walkers.empty()) return GM_OK;
  return hip_rc(launch_batch_values(reinterpret_cast<const double* const*>(B->d_vals), (int32_t)B->walkers.size(),
                                    s_dev, V_dev, dVds_dev, B->stream));
}

}  // extern "C"
