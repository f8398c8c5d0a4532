/*
 * gpumetad -- the per-step metadynamics bias pipeline on one AMD MI355X (gfx950).
 *
 * What the pipeline computes (paper: Methods, "Metadynamics Method"):
 *   the biased potential U_b = U_0 + V_b, with V_b a sum of Gaussian hills
 *   deposited at visited CV values.  The interatomic potential U_0 is not
 *   computed here: its forces arrive as an array, and the library adds the bias
 *   forces -dV_b/dx to it, which is the job the paper's GPUMD interface does each
 *   MD step (Results, "Frameworks of GPU-MetaD": the interface extracts the MD
 *   state, computes CVs and bias-driven forces on the GPU, and returns them).
 *
 * One context (gm_ctx) holds one system of N atoms, its cell and neighbour
 * lists, the per-atom intermediates of the collective variables, and the
 * device-resident hill history.  A timed MD step is
 *
 *     gm_cv_forward -> gm_bias_eval -> gm_cv_backward -> gm_apply_bias_forces
 *
 * with gm_build_neighbors every few steps and gm_deposit_hill at the
 * deposition pace.  Every call validates its arguments on the host, ENQUEUES
 * its kernels on the context's HIP stream and returns; none synchronises except
 * the calls marked "synchronous", which wait for the context's stream only.
 * Scalars (s, V, dV/ds) stay in device memory, so a whole window of steps can
 * be captured in a HIP graph.
 *
 * Memory: the library's device buffers come from a stream-ordered pool of its
 * own (one per device, keeping up to 4 GiB cached between uses).  A released
 * buffer stays with the library (up to 16 GiB per device, in size classes of
 * four per power of two; beyond that the oldest go back to the pool): it is
 * handed out again to an allocation on the stream it was released on, or on
 * another stream once the work before its release has completed.  Allocation
 * and release are operations on the stream the context or batch is bound to
 * at that moment, so creating and destroying them never waits for the device.
 *
 * Pointer conventions
 *   "dev"  : device memory (e.g. from hipMalloc), owned by the caller,
 *            read or written only by the enqueued kernels, never kept past the call.
 *   "host" : host memory, read or written before the call returns.
 *   Positions are always float32 [N][4] (x, y, z, w; w is ignored), 16-byte
 *   aligned, in the caller's atom order.  Force and gradient arrays are [N][4]
 *   of float32 (GM_FP32) or float64 (GM_FP64); their fourth lane is untouched.
 *   Lengths in Angstrom; energies in the unit of w0 and kBT (forces in
 *   energy/Angstrom).  The box is orthorhombic and periodic.
 *
 * Errors: every call returns GM_OK (0) or a negative GM_ERR_* code and never
 * throws.  Conditions only the device can see (neighbour overflow, a full hill
 * buffer, a non-finite CV, bias or force) set a sticky device error word that
 * gm_status() reads and clears.
 *
 * Threading: a context is not thread safe; use one context per stream.
 */
#ifndef GPUMETAD_H
#define GPUMETAD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------- */
#define GM_OK 0
#define GM_ERR_INVALID_ARG (-1)       /* null or misaligned pointer, bad size or parameter */
#define GM_ERR_OOM (-2)               /* a device allocation failed */
#define GM_ERR_HIP (-3)               /* a HIP runtime call or launch failed */
#define GM_ERR_BOX_TOO_SMALL (-4)     /* fewer than 3 cells of width >= r_c + skin on an axis */
#define GM_ERR_NEIGHBOR_OVERFLOW (-5) /* sticky: an atom has more than max_neighbors neighbours */
#define GM_ERR_HILL_CAPACITY (-6)     /* sticky: deposit into a full hill buffer */
#define GM_ERR_NONFINITE (-7)         /* sticky: NaN/Inf position, CV, bias or force */
#define GM_ERR_STATE (-8)             /* call order violated (see each call) */
#define GM_ERR_TOO_LARGE (-9)         /* size beyond the fixed scratch of an allocation-free call */

/* ---- collective variables ----------------------------------------------- */
/* GM_CV_COORD   s = (1/N) sum_i sum_{j: r_ij < r_c} 1/(1 + (r_ij/r0)^6)
 *               (the coordination number; paper, Results, GaN study).
 * GM_CV_Q6COUNT s = sum_i c_i, the smooth count of crystalline atoms from
 *               Steinhardt q6 (l = 6) bond order:
 *                 Q_i  = sum_{j: r_ij < r_c} f(r_ij) Y_6(r_hat_ij)  (13 reals)
 *                 d_ij = Q_i.Q_j / (|Q_i| |Q_j|)
 *                 n_i  = sum_j f(r_ij) / (1 + exp(-(d_ij - bond_d0)/bond_w))
 *                 c_i  = 1 / (1 + exp(-(n_i - count_n0)/count_w))
 *               with f = 1 below r_c - taper and a cosine taper to 0 at r_c.
 * GM_CV_COORD_Q6 the 2-D CV s = (s_COORD, s_Q6COUNT) over the same r_c.
 * GM_CV_EXTERNAL a context that holds only the hills of a CV the caller
 *               computes (params.dims components, e.g. the torsions or the
 *               nearest distance below): gm_bias_eval and gm_deposit_hill
 *               with an explicit s_dev, gm_hills_*, gm_fes_hills; the atom
 *               calls return GM_ERR_STATE and n_atoms may be 0.             */
#define GM_CV_COORD 1
#define GM_CV_Q6COUNT 2
#define GM_CV_COORD_Q6 3
#define GM_CV_EXTERNAL 4

#define GM_FP32 0
#define GM_FP64 1

typedef struct gm_params {
  int32_t cv_kind;       /* GM_CV_*                                           */
  int32_t precision;     /* GM_FP32 or GM_FP64 for the per-atom arithmetic;
                            global CV sums and all hill arithmetic are FP64   */
  double r_c;            /* CV cutoff, Angstrom                               */
  double skin;           /* Verlet skin: neighbour lists hold r < r_c + skin  */
  double taper;          /* q6 weight taper width (0 < taper <= r_c)          */
  double cn_r0;          /* coordination switch length r0                     */
  double bond_d0, bond_w;   /* bond sigmoid centre and width (q6 dot)         */
  double count_n0, count_w; /* count sigmoid centre and width (bonds)         */
  double sigma[2];       /* Gaussian hill widths per CV dimension             */
  double w0;             /* initial hill height                               */
  double gamma;          /* well-tempered bias factor (> 1); 0 = plain metad  */
  double kBT;            /* k_B T in the energy unit of w0                    */
  int64_t hill_capacity; /* maximum number of hills kept on the device        */
  int32_t max_neighbors; /* neighbour-list row width (rounded up to 4)        */
  int32_t brick[3];      /* cells per brick and axis (1..4); 0 = chosen per build */
  int32_t lds_kb;        /* LDS staging budget per workgroup in KiB; 0 = auto */
  double period[2];      /* period of each CV dimension (e.g. 2 pi for an angle);
                            hill distances use the nearest periodic image;
                            0 = not periodic                                  */
  int32_t dims;          /* CV dimensions of a GM_CV_EXTERNAL context (1 or 2);
                            ignored by the other kinds                        */
  int32_t tpa;           /* lanes that share one atom's neighbour rows in the
                            CV passes (1, 2 or 4); 0 = chosen per build       */
} gm_params;

typedef struct gm_ctx gm_ctx;

/* Create a context for n_atoms atoms whose kernels run on hip_stream
 * (a HIP stream handle; NULL = the null stream), on the current device.
 * Allocates and zero-fills every buffer the steps need, in order on
 * hip_stream (no wait).  *out is set to NULL on failure. */
int gm_create(gm_ctx** out, const gm_params* params, int64_t n_atoms, void* hip_stream);

/* Release everything the context owns, in stream order on the context's
 * stream (no wait): work already enqueued there may still use the buffers, and
 * work on other streams that uses them must be ordered before this call.  The
 * stream must still exist.  The buffers go back to the library's cache of
 * released device memory (see Memory above), not to the system. */
int gm_destroy(gm_ctx* ctx);

/* Re-bind the context to another stream (e.g. a capture stream).  The caller
 * orders the new stream after the context's work on the old one (an event),
 * as for any data the two share. */
int gm_set_stream(gm_ctx* ctx, void* hip_stream);

/* Build the cell list (a stable counting sort of atoms by cell, cells of
 * width >= r_c + skin) and the full neighbour lists
 *   N(i) = { j != i : |mic(x_j - x_i)|^2 < (r_c + skin)^2 }
 * with the distance test done in FP64 on the FP32 positions, no FMA.
 * pos4: dev float32 [N][4].  box: host double[3] (Lx, Ly, Lz).
 * Returns GM_ERR_BOX_TOO_SMALL if any axis holds fewer than 3 cells.
 * Rows hold at most max_neighbors entries; a longer row sets the sticky
 * GM_ERR_NEIGHBOR_OVERFLOW (grow with gm_reserve_neighbors and rebuild). */
int gm_build_neighbors(gm_ctx* ctx, const float* pos4, const double* box);

/* Evaluate the CV at pos4 (dev float32 [N][4], the same atoms as the last
 * build, moved by less than skin/2).  s_dev: dev double[dims], written.
 * GM_ERR_STATE before the first gm_build_neighbors. */
int gm_cv_forward(gm_ctx* ctx, const float* pos4, double* s_dev);

/* Bias and its CV gradient over the hills on the device
 * (paper, Methods: V_b(s) = sum_tau w_tau exp(-(s - s_tau)^2 / (2 sigma^2)),
 *  one Gaussian factor per CV dimension):
 *   V = sum_k h_k exp(-sum_d (s_d - c_kd)^2 / (2 sigma_d^2))
 *   dV/ds_d = -sum_k h_k exp(...) (s_d - c_kd) / sigma_d^2
 * s_dev: dev double[dims] (read).  V_dev: dev double[1], dVds_dev: dev
 * double[dims] (written; either may be NULL).  FP64 throughout; zero hills
 * give V = 0. */
int gm_bias_eval(gm_ctx* ctx, const double* s_dev, double* V_dev, double* dVds_dev);

/* Adjoint of the last gm_cv_forward, whose pos4 pointer it must be given
 * again (GM_ERR_STATE otherwise; the kernels work from the positions that
 * forward pass gathered, so the array must not have changed).  Computes the per-atom
 * adjoint state the force pass needs.  If grad4 != NULL it also writes
 *   grad4[i] = sum_d seed_d ds_d/dx_i
 * (dev [N][4] of the context precision, caller's atom order; lane 3 is left
 * alone).  seed_dev: dev double[dims], read only when grad4 != NULL; NULL
 * means seed 1 and is allowed with grad4 only when dims == 1.  GM_ERR_STATE
 * if no gm_cv_forward since the last build. */
int gm_cv_backward(gm_ctx* ctx, const float* pos4, const double* seed_dev, void* grad4);

/* Add the bias force to force4 in place (dev [N][4] of the context precision,
 * caller's atom order):
 *   F_i <- F_i - sum_d dV/ds_d * ds_d/dx_i       (from U_b = U_0 + V_b)
 * dVds_dev: dev double[dims], e.g. from gm_bias_eval.  GM_ERR_STATE unless
 * gm_cv_backward ran since the last gm_cv_forward, or if pos4 is not the
 * pointer that forward pass was given (the force is that of its positions). */
int gm_apply_bias_forces(gm_ctx* ctx, const float* pos4, const double* dVds_dev, void* force4);

/* Deposit one hill at s_dev (dev double[dims]) with the well-tempered height
 *   h = w0 exp(-V(s) / (kBT (gamma - 1)))     (gamma == 0: h = w0)
 * where V(s) is the bias of the hills already deposited (Barducci, Bussi,
 * Parrinello 2008; the paper names well-tempered metadynamics for its
 * rutile study).  s_dev == NULL deposits at the CV value of the context's
 * last forward pass (GM_ERR_STATE if there was none).  The hill count lives on the device, so the call can be
 * replayed inside a graph; a full buffer sets the sticky GM_ERR_HILL_CAPACITY
 * and deposits nothing. */
int gm_deposit_hill(gm_ctx* ctx, const double* s_dev);

/* Checkpoint the hill history (synchronous: waits for the context's stream).
 * centres: host double[cap*dims], heights: host double[cap]; *k receives the
 * hill count.  Either array may be NULL to query the count only.
 * GM_ERR_INVALID_ARG if cap < count. */
int gm_hills_get(gm_ctx* ctx, double* centres, double* heights, int64_t cap, int64_t* k);

/* Restore a hill history (synchronous: enqueued, then waits for the context's
 * stream so that the host arrays may be reused on return).
 * centres: host double[k*dims], heights: host double[k],
 * 0 <= k <= hill_capacity.  Bias sums run in hill index order, so a restored
 * history reproduces V bit for bit. */
int gm_hills_set(gm_ctx* ctx, const double* centres, const double* heights, int64_t k);

/* gm_hills_set from device arrays, enqueued and not waited for: centres_dev
 * dev double[k*dims], heights_dev dev double[k] (read by the copies on the
 * context's stream; keep them alive until that work has run).  For callers
 * that admit walkers while others run on the device (a serving loop) and so
 * must not block on a host copy. */
int gm_hills_set_device(gm_ctx* ctx, const double* centres_dev, const double* heights_dev, int64_t k);

/* Enqueue a copy of the sticky device error word (not cleared) into dst:
 * device memory or page-locked host memory (a pageable destination makes the
 * copy wait).  Once the stream has passed this point, gm_status_decode(*dst)
 * gives the GM_* code gm_status would return, without a synchronisation. */
int gm_status_copy(gm_ctx* ctx, int32_t* dst);
int gm_status_decode(int32_t word);

/* Read and clear the sticky device error word.  sync != 0 waits for the
 * stream first (synchronous); sync == 0 returns the code seen at the last
 * synchronous check without touching the device. */
int gm_status(gm_ctx* ctx, int sync);

/* Text for a GM_* code (static storage). */
const char* gm_strerror(int code);

/* Largest row length and total entries of the last neighbour build, and the
 * number of ordered pairs inside r_c at the last gm_cv_forward (0 before the
 * first one).  Any output pointer may be NULL (synchronous). */
int gm_neighbor_stats(gm_ctx* ctx, int32_t* max_count, int64_t* total, int64_t* cutoff_pairs);

/* Release the per-atom q6 rows of the context (the q-hat rows the forward
 * pass writes and the adjoint rows of gm_cv_backward: 2 x 16 values per atom
 * of the context precision) back to the library's pool, in stream order (no
 * wait); the next gm_cv_forward (or batch step) allocates them again.  For a
 * caller that recomputes the forward pass before each backward (the
 * differentiation's "recompute" mode: paper, Results, "Frameworks of
 * GPU-MetaD", forces by differentiating the CV), so that the context holds
 * no per-atom CV state between calls.  Backward and the force pass then need
 * a new gm_cv_forward (GM_ERR_STATE otherwise).  No effect on a coordination
 * context, which has no such rows. */
int gm_release_rows(gm_ctx* ctx);

/* Bytes of device memory the context holds now (its buffers in the pool;
 * host value, no device work). */
int gm_device_bytes(gm_ctx* ctx, int64_t* bytes);

/* Set the neighbour-list row width (rounded up to a multiple of 4) and
 * reallocate in stream order (no wait); the lists must be rebuilt afterwards. */
int gm_reserve_neighbors(gm_ctx* ctx, int32_t max_neighbors);

/* Copy the cell list of the last build (enqueued device-to-device copies):
 * perm_dev: dev int32[N], the atom ids in sorted (cell, atom) order;
 * cell_start_dev: dev int32[ncells + 1] (may be NULL); ncell: host int32[3]. */
int gm_copy_cell_list(gm_ctx* ctx, int32_t* perm_dev, int32_t* cell_start_dev, int32_t* ncell);

/* Copy the neighbour lists (enqueued): nbr_dev dev int32[N][row_width] whose
 * row t lists the sorted positions (indices into perm) of the neighbours of
 * the atom perm[t]; cnt_dev dev int32[N], the true row lengths;
 * row_width: host int32. */
int gm_copy_neighbors(gm_ctx* ctx, int32_t* nbr_dev, int32_t* cnt_dev, int32_t* row_width);

/* Per-atom values of the last gm_cv_forward, caller's atom order, written as
 * dev double[N] (enqueued):
 *   GM_ATOM_Q6  Steinhardt q6_i = sqrt(4 pi/13) |Q_i| / sum_j f(r_ij)
 *   GM_ATOM_NB  n_i, the weighted count of crystal-like bonds
 *   GM_ATOM_C   c_i, the crystalline indicator
 *   GM_ATOM_CN  sum_j 1/(1 + (r_ij/r0)^6), the per-atom coordination     */
#define GM_ATOM_Q6 1
#define GM_ATOM_NB 2
#define GM_ATOM_C 3
#define GM_ATOM_CN 4
int gm_atom_values(gm_ctx* ctx, int what, double* dst_dev);

/* ---- batches of walkers --------------------------------------------------
 * Many independent systems ("walkers", one context each, uneven sizes, any CV
 * kind) advanced together: every pass of the step is ONE launch for all
 * walkers of a CV kind, driven by a device table of per-walker arguments.
 * Each walker keeps its own lists, hills, tickets and partial sums, so its
 * results are bitwise the same as when it is stepped alone.  Walkers must
 * share the precision.  The batch re-binds every walker to its stream. */
typedef struct gm_batch gm_batch;

/* walkers: host array of count contexts; pos4 / force4: host arrays of count
 * device pointers (float32 [N_w][4] positions, [N_w][4] forces of the context
 * precision) that stay valid while the batch exists. */
int gm_batch_create(gm_batch** out, gm_ctx* const* walkers, int32_t count, const float* const* pos4,
                    void* const* force4, void* hip_stream);

/* Free the batch's device tables in stream order on its stream (no wait); the
 * walkers stay bound to that stream. */
int gm_batch_destroy(gm_batch* batch);

/* Replace the batch's members (same argument meaning as gm_batch_create;
 * count may be 0).  The batch keeps its device tables (grown only when a
 * larger member list needs it) and the table entries of the walkers that
 * stay, so a serving loop whose active set changes every few steps neither
 * frees nor reallocates device memory per change.  A context must be removed
 * by an update (or the batch destroyed) before the context is destroyed.
 * On GM_ERR_INVALID_ARG the batch keeps its previous members; on GM_ERR_OOM
 * or GM_ERR_HIP it is left with none.  Every member must have the batch's
 * precision; new members are bound to its stream. */
int gm_batch_update(gm_batch* batch, gm_ctx* const* walkers, int32_t count, const float* const* pos4,
                    void* const* force4);

/* Rebuild every walker's cell and neighbour lists; boxes: host double[count][3]. */
int gm_batch_build(gm_batch* batch, const double* boxes);

/* Rebuild the lists of some members: which = host array of count distinct
 * member indices (the order of the last create or update), boxes = host
 * double[count][3] (row i is the box of walker which[i]).  Walkers whose cell
 * grid and brick count each fit one workgroup's scan (at most 16,384) are
 * rebuilt together, one launch per stage of the rebuild; the others as
 * gm_build_neighbors does.  Lists and sorted order are bitwise those of
 * gm_build_neighbors.  Enqueued on hip_stream (NULL: the batch's stream); on
 * another stream the caller orders the work (that stream waits for the
 * batch's stream before the call, and the batch's stream for it after).
 * Buffers that must grow are allocated in the order of that stream.
 * GM_ERR_INVALID_ARG for an index out of range or repeated; box errors as in
 * gm_build_neighbors. */
int gm_batch_build_some(gm_batch* batch, const int32_t* which, int32_t count, const double* boxes,
                        void* hip_stream);

/* One MD step of the bias pipeline for every walker: CV forward, bias,
 * adjoint and F -= dV/ds ds/dx, each pass one launch per CV kind.  V and dV/ds
 * stay in the walker's context.  GM_ERR_STATE if a walker was never built. */
int gm_batch_step(gm_batch* batch);

/* Deposit one well-tempered hill per walker at its current CV value. */
int gm_batch_deposit(gm_batch* batch);

/* The same for some walkers only (each deposit as gm_deposit_hill would make
 * it, bitwise): which = host array of count distinct member indices (the
 * order of the last create or update); two launches per 64 walkers.
 * GM_ERR_INVALID_ARG for an index out of range or repeated, GM_ERR_STATE for a
 * walker not yet stepped (no CV value to deposit at). */
int gm_batch_deposit_some(gm_batch* batch, const int32_t* which, int32_t count);

/* Copy each walker's CV, bias and bias gradient of its last step (enqueued):
 * s_dev dev double[count][2] (second column 0 for 1-D CVs), V_dev dev
 * double[count], dVds_dev dev double[count][2] (second column 0 for 1-D
 * CVs); any may be NULL. */
int gm_batch_values(gm_batch* batch, double* s_dev, double* V_dev, double* dVds_dev);

/* Library version string. */
/* ---- CVs of a few atoms ----------------------------------------------------
 * Context-free calls enqueued on hip_stream (NULL = the null stream), FP64 on
 * the FP32 coordinates pos4 (dev float32 [n_atoms][4]) with the minimum image
 * in the orthorhombic box (host double[3]).  Index arrays live on the device;
 * an index outside [0, n_atoms) makes the CV it belongs to NaN and adds no
 * force (it is never dereferenced).  force4 is dev [n_atoms][4] of the given
 * precision (GM_FP32 / GM_FP64), caller's atom order, updated in place with
 *   F_i <- F_i - sum dV/ds . ds/dx_i
 * The CV values feed a GM_CV_EXTERNAL context (gm_bias_eval, gm_deposit_hill
 * with explicit s_dev; period 2 pi for an angle). */

/* Torsion angles of count atom quadruples (paper, Results, "Alanine
 * dipeptide torsion": Phi(C-N-CA-C) and Psi(N-CA-C-N)), IUPAC sign:
 *   b1 = x2 - x1, b2 = x3 - x2, b3 = x4 - x3,
 *   phi = atan2(|b2| b1.(b2 x b3), (b1 x b2).(b2 x b3))  in (-pi, pi].
 * quads_dev: dev int32[count][4]; phi_dev: dev double[count] (written).
 * 0 <= count <= 65536. */
int gm_torsions(const float* pos4, int64_t n_atoms, const int32_t* quads_dev, int32_t count, const double* box,
                double* phi_dev, void* hip_stream);

/* Torsion bias forces with dVdphi_dev (dev double[count]); the torsions are
 * summed one after another, so atoms shared by several torsions get a fixed
 * order. */
int gm_torsion_forces(const float* pos4, int64_t n_atoms, const int32_t* quads_dev, int32_t count, const double* box,
                      const double* dVdphi_dev, void* force4, int32_t precision, void* hip_stream);

/* Distance from atom centre to the nearest atom of a set (paper, Results,
 * "Water dissociation on rutile (110) surface": a surface oxygen and its
 * nearest hydrogen):  s = min_{j in set, j != centre} |mic(x_j - x_centre)|,
 * ties to the earliest member.  members_dev: dev int32[count], count >= 1;
 * s_dev: dev double[1]; nearest_dev: dev int32[1] or NULL (the atom). */
int gm_nearest_distance(const float* pos4, int64_t n_atoms, int32_t centre, const int32_t* members_dev,
                        int32_t count, const double* box, double* s_dev, int32_t* nearest_dev, void* hip_stream);

/* Its bias force: F_centre += dV/ds u, F_nearest -= dV/ds u, u the unit
 * vector from the centre to the nearest atom (dVds_dev: dev double[1]). */
int gm_nearest_distance_forces(const float* pos4, int64_t n_atoms, int32_t centre, const int32_t* members_dev,
                               int32_t count, const double* box, const double* dVds_dev, void* force4,
                               int32_t precision, void* hip_stream);

/* Lattice parameters as CVs (paper, Results, "B4-B1 phase transition":
 * the triaxial lattice parameters of an NPT run): s = (L_x, L_y, L_z)[:dims]
 * need no kernel; the bias acts on the cell through the virial the barostat
 * adds, W_aa = -L_a dV/dL_a (host arrays of dims <= 3 values). */
int gm_lattice_virial(const double* box, const double* dVdL, int32_t dims, double* virial);

/* ---- free energy ------------------------------------------------------------
 * Reweighting of a biased run (paper, Methods: P(s) = <delta(s - s(R))
 * e^{beta V}> / <e^{beta V}> over the biased ensemble, F = -(1/beta) log P).
 * Samples s_dev dev double[T][dims] and V_dev dev double[T] (the bias at each
 * sample); bins i_d = floor((s_d - lo_d) / w_d), w_d = (hi_d - lo_d)/nbins_d,
 * bin id i_0 + nbins_0 i_1; samples off the grid count in the denominator
 * only.  F_dev: dev double[prod nbins] (written), -kBT log P per bin, +inf
 * where no sample fell.  The per-bin sums use FP64 atomics: reproducible to
 * about 1e-15 relative, not bit for bit.  Host lo, hi (double[dims]), nbins
 * (int32[dims]); dims 1 or 2; at most 2^24 bins.  Temporary device memory
 * comes from the stream-ordered allocator. */
int gm_fes_reweight(const double* s_dev, const double* V_dev, int64_t T, int32_t dims, const double* lo,
                    const double* hi, const int32_t* nbins, double kBT, double* F_dev, void* hip_stream);

/* gm_fes_reweight for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops that forbid allocation): the same kernels,
 * arguments and results, with the per-workgroup partials and per-bin sums in
 * a fixed scratch array of the library (about 530 KiB per device, held from
 * the first call on a device until the process ends) instead of the
 * stream-ordered allocator.  No device memory is allocated or freed.
 * At most 65536 bins (prod nbins); a larger grid returns GM_ERR_TOO_LARGE
 * before any device work.  Every call on one device shares its scratch:
 * calls that overlap on a device (on different streams, or from different
 * threads without ordering) race and give wrong results; calls ordered on one
 * stream are safe, since each call overwrites the scratch before reading it. */
int gm_fes_reweight_noalloc(const double* s_dev, const double* V_dev, int64_t T, int32_t dims, const double* lo,
                            const double* hi, const int32_t* nbins, double kBT, double* F_dev, void* hip_stream);

/* The free energy from the context's hills on the grid of bin centres
 * (lo_d + (i_d + 1/2) w_d): F = -V (plain metadynamics) or
 * F = -gamma/(gamma - 1) V (well-tempered), hills summed in index order.
 * Same grid arguments and F_dev layout as gm_fes_reweight (dims = the
 * context's). */
int gm_fes_hills(gm_ctx* ctx, const double* lo, const double* hi, const int32_t* nbins, double* F_dev);

const char* gm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GPUMETAD_H */
