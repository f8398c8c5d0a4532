/*
 * Plain FP64 CPU oracle for the per-step metadynamics bias pipeline.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no source with the HIP path.
 *
 * Everything here is single threaded, double precision, and written as the
 * definition of each quantity, in the order the method states it:
 *
 *  - the biased potential U_b = U_0 + V_b and the Gaussian-hill bias
 *    V_b(s) = sum_tau w_tau exp(-(s - s_tau)^2 / (2 sigma^2))
 *    (paper, Methods, "Metadynamics Method", the equations for U_b and V_b);
 *  - well-tempered hill heights (named in the paper's rutile study; the
 *    standard form w = w0 exp(-V(s)/(k_B T (gamma-1))) of Barducci, Bussi and
 *    Parrinello, PRL 100, 020603 (2008));
 *  - the coordination-number CV (named for the GaN study in the paper,
 *    Results, "B4-B1 phase transition"), rational switch 1/(1+(r/r0)^6);
 *  - the Steinhardt q6 crystalline-atom count (Steinhardt, Nelson, Ronchetti,
 *    PRB 28, 784 (1983) for q6; the bond/count sigmoids are the workload's
 *    definition of the CV);
 *  - the bias force F <- F - dV/ds . ds/dx, obtained from U_b (Methods) by the
 *    chain rule.  The paper gets it from autodiff (Results, "Frameworks of
 *    GPU-MetaD"); here it is plain reverse-mode differentiation written out as
 *    a scatter over pairs, with no use of the symmetries the GPU path exploits.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no FMA contraction, so the
 * FP64 pair test and cell binning round exactly as written).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define GMO_OK 0
#define GMO_BOX_TOO_SMALL (-4)
#define GMO_INVALID (-1)

/* ------------------------------------------------------------------------ */
/* Orthorhombic periodic box: minimum image and squared distance.           */
/* d = x_j - x_i; d_a -= L_a * rint(d_a / L_a)  (rint: ties to even).       */
/* r^2 = (dx*dx + dy*dy) + dz*dz, left to right, no fused multiply-add.     */
/* ------------------------------------------------------------------------ */
static void min_image(const double *xi, const double *xj, const double box[3],
                      double d[3]) {
  for (int a = 0; a < 3; a++) {
    double v = xj[a] - xi[a];
    d[a] = v - box[a] * rint(v / box[a]);
  }
}

static double sq_dist(const double d[3]) {
  return d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
}

/* ------------------------------------------------------------------------ */
/* Cell list: a counting sort of atoms by cell id.                          */
/* n_a = floor(L_a / r_list), at least 3 per axis.                          */
/* w = x - L floor(x/L); c_a = clamp(floor(w_a * (n_a / L_a)), 0, n_a - 1); */
/* id = (c_z n_y + c_y) n_x + c_x.  Sorted order: ascending (cell, atom).   */
/* ------------------------------------------------------------------------ */
int gmo_cell_grid(const double box[3], double r_list, int32_t ncell[3]) {
  if (!(r_list > 0.0)) return GMO_INVALID;
  for (int a = 0; a < 3; a++) {
    double n = floor(box[a] / r_list);
    if (n < 3.0) return GMO_BOX_TOO_SMALL;
    if (n > 1.0e6) return GMO_INVALID;
    ncell[a] = (int32_t)n;
  }
  return GMO_OK;
}

void gmo_cell_ids(const double *pos, int64_t n, const double box[3],
                  const int32_t ncell[3], int32_t *cell) {
  double inv[3];
  for (int a = 0; a < 3; a++) inv[a] = (double)ncell[a] / box[a];
  for (int64_t i = 0; i < n; i++) {
    int32_t c[3];
    for (int a = 0; a < 3; a++) {
      double x = pos[3 * i + a];
      double w = x - box[a] * floor(x / box[a]);
      double f = floor(w * inv[a]);
      if (f < 0.0) f = 0.0;
      if (f > (double)(ncell[a] - 1)) f = (double)(ncell[a] - 1);
      c[a] = (int32_t)f;
    }
    cell[i] = (c[2] * ncell[1] + c[1]) * ncell[0] + c[0];
  }
}

/* Stable counting sort: counts, exclusive prefix sum, scatter in atom order. */
void gmo_cell_sort(const int32_t *cell, int64_t n, int64_t ncells,
                   int32_t *perm, int32_t *cell_start) {
  int64_t *fill = (int64_t *)calloc((size_t)ncells, sizeof(int64_t));
  for (int64_t c = 0; c <= ncells; c++) cell_start[c] = 0;
  for (int64_t i = 0; i < n; i++) cell_start[cell[i] + 1] += 1;
  for (int64_t c = 0; c < ncells; c++) cell_start[c + 1] += cell_start[c];
  for (int64_t i = 0; i < n; i++) {
    int32_t c = cell[i];
    perm[cell_start[c] + fill[c]] = (int32_t)i;
    fill[c] += 1;
  }
  free(fill);
}

/* ------------------------------------------------------------------------ */
/* Neighbour sets N(i) = { j != i : r_ij^2 < r_list^2 }  (full lists, CSR,  */
/* each row ascending in j).  Returns the total number of entries; if it    */
/* exceeds cap only the offsets are written.                                */
/* ------------------------------------------------------------------------ */
int64_t gmo_neighbors_brute(const double *pos, int64_t n, const double box[3],
                            double r_list, int64_t *offsets, int32_t *nbr,
                            int64_t cap) {
  double rl2 = r_list * r_list;
  int64_t total = 0;
  offsets[0] = 0;
  for (int64_t i = 0; i < n; i++) {
    for (int64_t j = 0; j < n; j++) {
      if (j == i) continue;
      double d[3];
      min_image(&pos[3 * i], &pos[3 * j], box, d);
      if (sq_dist(d) < rl2) {
        if (total < cap) nbr[total] = (int32_t)j;
        total++;
      }
    }
    offsets[i + 1] = total;
  }
  return total;
}

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/* Same sets, found through the cell list (27-cell stencil, periodic). */
int64_t gmo_neighbors_cells(const double *pos, int64_t n, const double box[3],
                            double r_list, int64_t *offsets, int32_t *nbr,
                            int64_t cap) {
  int32_t nc[3];
  if (gmo_cell_grid(box, r_list, nc) != GMO_OK) return -1;
  int64_t ncells = (int64_t)nc[0] * nc[1] * nc[2];
  int32_t *cell = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int32_t *start = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ncells + 1));
  gmo_cell_ids(pos, n, box, nc, cell);
  gmo_cell_sort(cell, n, ncells, perm, start);
  double rl2 = r_list * r_list;
  int64_t total = 0;
  offsets[0] = 0;
  for (int64_t i = 0; i < n; i++) {
    int32_t c = cell[i];
    int32_t cx = c % nc[0], cy = (c / nc[0]) % nc[1], cz = c / (nc[0] * nc[1]);
    int64_t row0 = total;
    for (int dz = -1; dz <= 1; dz++)
      for (int dy = -1; dy <= 1; dy++)
        for (int dx = -1; dx <= 1; dx++) {
          int32_t x = (cx + dx + nc[0]) % nc[0];
          int32_t y = (cy + dy + nc[1]) % nc[1];
          int32_t z = (cz + dz + nc[2]) % nc[2];
          int32_t cc = (z * nc[1] + y) * nc[0] + x;
          for (int32_t k = start[cc]; k < start[cc + 1]; k++) {
            int32_t j = perm[k];
            if (j == i) continue;
            double d[3];
            min_image(&pos[3 * i], &pos[3 * j], box, d);
            if (sq_dist(d) < rl2) {
              if (total < cap) nbr[total] = j;
              total++;
            }
          }
        }
    if (total <= cap) qsort(&nbr[row0], (size_t)(total - row0), sizeof(int32_t), cmp_i32);
    offsets[i + 1] = total;
  }
  free(cell);
  free(perm);
  free(start);
  return total;
}

/* ------------------------------------------------------------------------ */
/* Coordination number (mean over atoms, every ordered pair counted):        */
/*   s_CN = (1/N) sum_i sum_{j in N(i), r_ij < r_c} sw(r_ij)                 */
/*   sw(r) = (1 - x^6)/(1 - x^12) = 1/(1 + x^6),  x = r/r0                   */
/*   sw'(r) = -6 x^5 / (r0 (1 + x^6)^2)                                      */
/* ------------------------------------------------------------------------ */
static double cn_switch(double r, double r0, double *dsw) {
  double x = r / r0;
  double x5 = x * x * x * x * x;
  double x6 = x5 * x;
  double den = 1.0 + x6;
  if (dsw) *dsw = -6.0 * x5 / (r0 * den * den);
  return 1.0 / den;
}

double gmo_cn_forward(const double *pos, int64_t n, const double box[3],
                      const int64_t *offsets, const int32_t *nbr, double r0,
                      double r_c, double *cn_atom) {
  double total = 0.0;
  for (int64_t i = 0; i < n; i++) {
    double ci = 0.0;
    for (int64_t k = offsets[i]; k < offsets[i + 1]; k++) {
      double d[3];
      min_image(&pos[3 * i], &pos[3 * nbr[k]], box, d);
      double r = sqrt(sq_dist(d));
      if (r < r_c) ci += cn_switch(r, r0, NULL);
    }
    if (cn_atom) cn_atom[i] = ci;
    total += ci;
  }
  return total / (double)n;
}

/* ds_CN/dx by reverse mode, scattering each ordered pair onto both atoms. */
void gmo_cn_gradient(const double *pos, int64_t n, const double box[3],
                     const int64_t *offsets, const int32_t *nbr, double r0,
                     double r_c, double *dsdx) {
  memset(dsdx, 0, sizeof(double) * 3 * (size_t)n);
  for (int64_t i = 0; i < n; i++) {
    for (int64_t k = offsets[i]; k < offsets[i + 1]; k++) {
      int64_t j = nbr[k];
      double d[3];
      min_image(&pos[3 * i], &pos[3 * j], box, d);
      double r = sqrt(sq_dist(d));
      if (!(r < r_c)) continue;
      double dsw;
      cn_switch(r, r0, &dsw);
      double rbar = dsw / (double)n; /* ds/dr_ij for this ordered pair */
      for (int a = 0; a < 3; a++) {
        double t = rbar * d[a] / r; /* dr/dx_j = +d/r, dr/dx_i = -d/r */
        dsdx[3 * j + a] += t;
        dsdx[3 * i + a] -= t;
      }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Spherical harmonics Y_6m, orthonormal, Condon-Shortley phase.             */
/*   P_6 from Rodrigues' formula  P_l(z) = 1/(2^l l!) d^l/dz^l (z^2 - 1)^l   */
/*   D_m(z) = d^m P_6 / dz^m                                                 */
/*   Y_6m(u) = K_m (-1)^m D_m(z) (x + i y)^m,  m >= 0, u = (x, y, z) unit    */
/*   K_m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)                                 */
/*   Y_6,-m = (-1)^m conj(Y_6m)                                              */
/* Real 13-vector: v = (Y_60, sqrt2 Re Y_61, sqrt2 Im Y_61, ...,             */
/*   sqrt2 Re Y_66, sqrt2 Im Y_66), so v_i . v_j = sum_m q_im conj(q_jm).    */
/* ------------------------------------------------------------------------ */
static double fact(int k) {
  double f = 1.0;
  for (int i = 2; i <= k; i++) f *= (double)i;
  return f;
}

static double binom(int n, int k) { return fact(n) / (fact(k) * fact(n - k)); }

/* dcoef[m][p] = coefficient of z^p in D_m(z), m = 0..7 (D_7 = 0). */
static double dcoef[8][7];
static double kconst[7];
static int tables_ready = 0;

static void make_tables(void) {
  if (tables_ready) return;
  /* (z^2 - 1)^6 = sum_k C(6,k) z^(2k) (-1)^(6-k); degree 12. */
  double a[13] = {0};
  for (int k = 0; k <= 6; k++) a[2 * k] = binom(6, k) * ((6 - k) % 2 ? -1.0 : 1.0);
  /* Differentiate six times, divide by 2^6 6!. */
  double scale = 64.0 * fact(6);
  for (int p = 0; p <= 6; p++) dcoef[0][p] = a[p + 6] * fact(p + 6) / fact(p) / scale;
  for (int m = 1; m <= 7; m++)
    for (int p = 0; p <= 6; p++)
      dcoef[m][p] = (p + 1 <= 6) ? dcoef[m - 1][p + 1] * (double)(p + 1) : 0.0;
  for (int m = 0; m <= 6; m++)
    kconst[m] = sqrt(13.0 / (4.0 * M_PI) * fact(6 - m) / fact(6 + m));
  tables_ready = 1;
}

static double poly_eval(const double *c, double z) {
  double s = 0.0, zp = 1.0;
  for (int p = 0; p <= 6; p++) {
    s += c[p] * zp;
    zp *= z;
  }
  return s;
}

/* Integer power, so that zeta^0 = 1 exactly and no branch cut is involved. */
static double complex cipow(double complex z, int m) {
  double complex p = 1.0;
  for (int k = 0; k < m; k++) p *= z;
  return p;
}

/* Complex Y_6m for m = 0..6 at unit vector u. */
void gmo_ylm6_complex(const double u[3], double *re, double *im) {
  make_tables();
  double complex zeta = u[0] + I * u[1];
  for (int m = 0; m <= 6; m++) {
    double complex y = kconst[m] * ((m % 2) ? -1.0 : 1.0) *
                       poly_eval(dcoef[m], u[2]) * cipow(zeta, m);
    re[m] = creal(y);
    im[m] = cimag(y);
  }
}

/* Real 13-vector v(u) and, if jac != NULL, its Jacobian with respect to the
 * components of u treated as free variables: jac[a*3 + b] = dv_a / du_b.      */
static void ylm6_real(const double u[3], double v[13], double *jac) {
  make_tables();
  double complex zeta = u[0] + I * u[1];
  const double sq2 = sqrt(2.0);
  for (int m = 0; m <= 6; m++) {
    double pre = kconst[m] * ((m % 2) ? -1.0 : 1.0);
    double dm = poly_eval(dcoef[m], u[2]);
    double dm1 = poly_eval(dcoef[m + 1], u[2]);
    double complex y = pre * dm * cipow(zeta, m);
    double complex yx = (m > 0) ? pre * dm * (double)m * cipow(zeta, m - 1) : 0.0;
    double complex yy = I * yx;
    double complex yz = pre * dm1 * cipow(zeta, m);
    if (m == 0) {
      v[0] = creal(y);
      if (jac) {
        jac[0] = creal(yx);
        jac[1] = creal(yy);
        jac[2] = creal(yz);
      }
    } else {
      int ar = 2 * m - 1, ai = 2 * m;
      v[ar] = sq2 * creal(y);
      v[ai] = sq2 * cimag(y);
      if (jac) {
        jac[3 * ar + 0] = sq2 * creal(yx);
        jac[3 * ar + 1] = sq2 * creal(yy);
        jac[3 * ar + 2] = sq2 * creal(yz);
        jac[3 * ai + 0] = sq2 * cimag(yx);
        jac[3 * ai + 1] = sq2 * cimag(yy);
        jac[3 * ai + 2] = sq2 * cimag(yz);
      }
    }
  }
}

void gmo_ylm6_real(const double u[3], double *v13) { ylm6_real(u, v13, NULL); }

/* ------------------------------------------------------------------------ */
/* q6 crystalline-atom count.                                                */
/*  f(r): 1 for r <= rc - D; (1 + cos(pi (r - rc + D)/D))/2 on (rc-D, rc);   */
/*        0 for r >= rc.   (D = taper width.)                                 */
/*  Q_i = sum_{j in N(i), r<rc} f(r_ij) v(r_hat_ij)        (13 reals)        */
/*  qhat_i = Q_i / |Q_i|   (qhat_i = 0 if |Q_i| < 1e-12)                     */
/*  d_ij = qhat_i . qhat_j;  b_ij = 1/(1 + exp(-(d_ij - d0)/w_b))            */
/*  n_i = sum_j f(r_ij) b_ij;  c_i = 1/(1 + exp(-(n_i - n0)/w_c))            */
/*  s = sum_i c_i   (summed in atom index order)                             */
/* ------------------------------------------------------------------------ */
typedef struct {
  double r_c, taper, bond_d0, bond_w, count_n0, count_w;
} gmo_q6_params;

static double taper_weight(double r, double rc, double D, double *df) {
  if (r <= rc - D) {
    *df = 0.0;
    return 1.0;
  }
  if (r < rc) {
    double t = M_PI * (r - rc + D) / D;
    *df = -0.5 * M_PI / D * sin(t);
    return 0.5 * (1.0 + cos(t));
  }
  *df = 0.0;
  return 0.0;
}

static double logistic(double x, double centre, double width, double *dydx) {
  double y = 1.0 / (1.0 + exp(-(x - centre) / width));
  if (dydx) *dydx = y * (1.0 - y) / width;
  return y;
}

static double dot13(const double *a, const double *b) {
  double s = 0.0;
  for (int k = 0; k < 13; k++) s += a[k] * b[k];
  return s;
}

/* Forward pass.  Any of the per-atom outputs may be NULL.                   */
double gmo_q6_forward(const double *pos, int64_t n, const double box[3],
                      const int64_t *offsets, const int32_t *nbr,
                      const gmo_q6_params *p, double *Q_out, double *qhat_out,
                      double *qnorm_out, double *nb_out, double *c_out,
                      double *dc_out, double *fsum_out) {
  double *Q = (double *)calloc((size_t)n * 13, sizeof(double));
  double *qhat = (double *)calloc((size_t)n * 13, sizeof(double));
  for (int64_t i = 0; i < n; i++) {
    double fsum = 0.0;
    for (int64_t k = offsets[i]; k < offsets[i + 1]; k++) {
      double d[3];
      min_image(&pos[3 * i], &pos[3 * nbr[k]], box, d);
      double r = sqrt(sq_dist(d));
      if (!(r < p->r_c)) continue;
      double df;
      double f = taper_weight(r, p->r_c, p->taper, &df);
      double u[3] = {d[0] / r, d[1] / r, d[2] / r};
      double v[13];
      ylm6_real(u, v, NULL);
      for (int a = 0; a < 13; a++) Q[13 * i + a] += f * v[a];
      fsum += f;
    }
    double qn = sqrt(dot13(&Q[13 * i], &Q[13 * i]));
    if (qn >= 1e-12)
      for (int a = 0; a < 13; a++) qhat[13 * i + a] = Q[13 * i + a] / qn;
    if (qnorm_out) qnorm_out[i] = qn;
    if (fsum_out) fsum_out[i] = fsum;
  }
  double s = 0.0;
  for (int64_t i = 0; i < n; i++) {
    double nb = 0.0;
    for (int64_t k = offsets[i]; k < offsets[i + 1]; k++) {
      int64_t j = nbr[k];
      double d[3];
      min_image(&pos[3 * i], &pos[3 * j], box, d);
      double r = sqrt(sq_dist(d));
      if (!(r < p->r_c)) continue;
      double df;
      double f = taper_weight(r, p->r_c, p->taper, &df);
      double b = logistic(dot13(&qhat[13 * i], &qhat[13 * j]), p->bond_d0, p->bond_w, NULL);
      nb += f * b;
    }
    double dc;
    double c = logistic(nb, p->count_n0, p->count_w, &dc);
    if (nb_out) nb_out[i] = nb;
    if (c_out) c_out[i] = c;
    if (dc_out) dc_out[i] = dc;
    s += c;
  }
  if (Q_out) memcpy(Q_out, Q, sizeof(double) * 13 * (size_t)n);
  if (qhat_out) memcpy(qhat_out, qhat, sizeof(double) * 13 * (size_t)n);
  free(Q);
  free(qhat);
  return s;
}

/* ds/dx for the q6 count, by reverse mode over the forward pass above.
 * Adjoints: nbar_i = c'_i; for each ordered pair (i,j) with r < rc:
 *   through f:  rbar = nbar_i f'(r_ij) b_ij          -> x_j += rbar r_hat, x_i -= rbar r_hat
 *   through d:  dbar = nbar_i f(r_ij) b'(d_ij)       -> qbar_i += dbar qhat_j, qbar_j += dbar qhat_i
 * Normalisation: Qbar_i = (qbar_i - (qhat_i.qbar_i) qhat_i) / |Q_i|.
 * Through Q: for each ordered pair (i,j), u = f(r) v(r_hat) with r = x_j - x_i:
 *   t = (du/dr)^T Qbar_i  -> x_j += t, x_i -= t
 * du/dr = f'(r) v r_hat^T + f(r) (dv/du)(I - r_hat r_hat^T)/r.              */
void gmo_q6_gradient(const double *pos, int64_t n, const double box[3],
                     const int64_t *offsets, const int32_t *nbr,
                     const gmo_q6_params *p, double *dsdx) {
  double *qhat = (double *)calloc((size_t)n * 13, sizeof(double));
  double *qnorm = (double *)calloc((size_t)n, sizeof(double));
  double *dc = (double *)calloc((size_t)n, sizeof(double));
  double *qbar = (double *)calloc((size_t)n * 13, sizeof(double));
  gmo_q6_forward(pos, n, box, offsets, nbr, p, NULL, qhat, qnorm, NULL, NULL, dc, NULL);
  memset(dsdx, 0, sizeof(double) * 3 * (size_t)n);
  for (int64_t i = 0; i < n; i++) {
    for (int64_t k = offsets[i]; k < offsets[i + 1]; k++) {
      int64_t j = nbr[k];
      double d[3];
      min_image(&pos[3 * i], &pos[3 * j], box, d);
      double r = sqrt(sq_dist(d));
      if (!(r < p->r_c)) continue;
      double df;
      double f = taper_weight(r, p->r_c, p->taper, &df);
      double db;
      double b = logistic(dot13(&qhat[13 * i], &qhat[13 * j]), p->bond_d0, p->bond_w, &db);
      double rbar = dc[i] * df * b;
      for (int a = 0; a < 3; a++) {
        dsdx[3 * j + a] += rbar * d[a] / r;
        dsdx[3 * i + a] -= rbar * d[a] / r;
      }
      double dbar = dc[i] * f * db;
      for (int a = 0; a < 13; a++) {
        qbar[13 * i + a] += dbar * qhat[13 * j + a];
        qbar[13 * j + a] += dbar * qhat[13 * i + a];
      }
    }
  }
  for (int64_t i = 0; i < n; i++) {
    double *qb = &qbar[13 * i];
    const double *qh = &qhat[13 * i];
    if (qnorm[i] < 1e-12) {
      for (int a = 0; a < 13; a++) qb[a] = 0.0;
      continue;
    }
    double proj = dot13(qh, qb);
    for (int a = 0; a < 13; a++) qb[a] = (qb[a] - proj * qh[a]) / qnorm[i];
  }
  for (int64_t i = 0; i < n; i++) {
    const double *Qb = &qbar[13 * i];
    for (int64_t k = offsets[i]; k < offsets[i + 1]; k++) {
      int64_t j = nbr[k];
      double d[3];
      min_image(&pos[3 * i], &pos[3 * j], box, d);
      double r = sqrt(sq_dist(d));
      if (!(r < p->r_c)) continue;
      double df;
      double f = taper_weight(r, p->r_c, p->taper, &df);
      double u[3] = {d[0] / r, d[1] / r, d[2] / r};
      double v[13], jac[39];
      ylm6_real(u, v, jac);
      /* du_a/dr_b = f' v_a u_b + (f/r) sum_c jac[a][c] (delta_cb - u_c u_b) */
      double t[3] = {0.0, 0.0, 0.0};
      for (int a = 0; a < 13; a++) {
        double ju = jac[3 * a + 0] * u[0] + jac[3 * a + 1] * u[1] + jac[3 * a + 2] * u[2];
        for (int b = 0; b < 3; b++) {
          double dudr = df * v[a] * u[b] + (f / r) * (jac[3 * a + b] - ju * u[b]);
          t[b] += Qb[a] * dudr;
        }
      }
      for (int b = 0; b < 3; b++) {
        dsdx[3 * j + b] += t[b];
        dsdx[3 * i + b] -= t[b];
      }
    }
  }
  free(qhat);
  free(qnorm);
  free(dc);
  free(qbar);
}

/* ------------------------------------------------------------------------ */
/* Gaussian-hill bias (Methods, the equation for V_b), dims-dimensional CV:  */
/*   V(s) = sum_k h_k exp(-sum_d (s_d - c_kd)^2 / (2 sigma_d^2))             */
/*   dV/ds_d = -sum_k h_k exp(...) (s_d - c_kd) / sigma_d^2                  */
/* Sums run in hill index order.                                             */
/* ------------------------------------------------------------------------ */
/* The distance of a CV value from a hill centre along dimension d.  A
 * periodic CV (period[d] > 0, e.g. a torsion angle with period 2 pi) uses the
 * nearest periodic image of the difference.                                 */
static double cv_delta(double s, double c, const double *period, int d) {
  double x = s - c;
  if (period && period[d] > 0.0) x -= period[d] * rint(x / period[d]);
  return x;
}

void gmo_bias(const double *centres, const double *heights, int64_t K, int dims,
              const double *sigma, const double *period, const double *s,
              double *V, double *dVds) {
  double v = 0.0;
  double g[8] = {0};
  for (int64_t k = 0; k < K; k++) {
    double arg = 0.0;
    for (int d = 0; d < dims; d++) {
      double x = cv_delta(s[d], centres[k * dims + d], period, d);
      arg += x * x / (2.0 * sigma[d] * sigma[d]);
    }
    double e = heights[k] * exp(-arg);
    v += e;
    for (int d = 0; d < dims; d++)
      g[d] += -e * cv_delta(s[d], centres[k * dims + d], period, d) /
              (sigma[d] * sigma[d]);
  }
  *V = v;
  if (dVds)
    for (int d = 0; d < dims; d++) dVds[d] = g[d];
}

/* Well-tempered height at a new centre given the bias V already there:
 *   h = w0 exp(-V / (k_B T (gamma - 1)));  gamma == 0 selects plain
 *   metadynamics (constant height w0).                                      */
double gmo_wt_height(double w0, double gamma, double kBT, double V) {
  if (gamma == 0.0) return w0;
  return w0 * exp(-V / (kBT * (gamma - 1.0)));
}

/* Deposit a sequence of hills in index order: height k uses hills 0..k-1.   */
void gmo_deposit_sequence(const double *centres, int64_t K, int dims,
                          const double *sigma, const double *period, double w0,
                          double gamma, double kBT, double *heights) {
  for (int64_t k = 0; k < K; k++) {
    double V;
    gmo_bias(centres, heights, k, dims, sigma, period, &centres[k * dims], &V,
             NULL);
    heights[k] = gmo_wt_height(w0, gamma, kBT, V);
  }
}

/* ------------------------------------------------------------------------ */
/* Torsion angle of four atoms, the CV pair (Phi, Psi) of the paper's        */
/* alanine dipeptide study (Results, "Alanine dipeptide torsion"), IUPAC     */
/* sign.  b1 = x2 - x1, b2 = x3 - x2, b3 = x4 - x3 (minimum images),          */
/* n1 = b1 x b2, n2 = b2 x b3:                                                */
/*   phi = atan2(|b2| b1.n2, n1.n2)   in (-pi, pi].                           */
/* Gradient: the end atoms move phi along the plane normals,                  */
/*   dphi/dx1 = -|b2|/|n1|^2 n1,   dphi/dx4 = |b2|/|n2|^2 n2,                 */
/* and with p = b1.b2/|b2|^2, q = b3.b2/|b2|^2 the middle atoms take          */
/*   dphi/dx2 = -(1 + p) dphi/dx1 + q dphi/dx4,                               */
/*   dphi/dx3 = -(1 + q) dphi/dx4 + p dphi/dx1                                */
/* (the four sum to zero: phi is invariant under translation).               */
/* ------------------------------------------------------------------------ */
static void cross3(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

void gmo_torsions(const double *pos, const double box[3], const int32_t *quads,
                  int64_t count, double *phi, double *grad) {
  for (int64_t t = 0; t < count; t++) {
    const int32_t *q = &quads[4 * t];
    double b1[3], b2[3], b3[3], n1[3], n2[3];
    min_image(&pos[3 * q[0]], &pos[3 * q[1]], box, b1);
    min_image(&pos[3 * q[1]], &pos[3 * q[2]], box, b2);
    min_image(&pos[3 * q[2]], &pos[3 * q[3]], box, b3);
    cross3(b1, b2, n1);
    cross3(b2, b3, n2);
    const double lb2 = sqrt(dot3(b2, b2));
    phi[t] = atan2(lb2 * dot3(b1, n2), dot3(n1, n2));
    if (!grad) continue;
    double *g = &grad[12 * t];
    const double n1n1 = dot3(n1, n1), n2n2 = dot3(n2, n2), b2b2 = lb2 * lb2;
    const double p = dot3(b1, b2) / b2b2, qq = dot3(b3, b2) / b2b2;
    for (int a = 0; a < 3; a++) {
      const double g1 = -lb2 / n1n1 * n1[a], g4 = lb2 / n2n2 * n2[a];
      g[0 + a] = g1;
      g[3 + a] = -(1.0 + p) * g1 + qq * g4;
      g[6 + a] = -(1.0 + qq) * g4 + p * g1;
      g[9 + a] = g4;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Distance from one atom to the nearest atom of a set (minimum image), the  */
/* CV of the paper's rutile study (Results, "Water dissociation on rutile    */
/* (110) surface": a surface oxygen and its nearest hydrogen).  Ties go to   */
/* the earliest member of the set; the centre itself is skipped.  The CV is  */
/* the distance of that pair, so ds/dx_centre = -u and ds/dx_nearest = u,    */
/* u the unit vector from the centre to the nearest atom.                    */
/* ------------------------------------------------------------------------ */
double gmo_nearest_distance(const double *pos, const double box[3],
                            int32_t centre, const int32_t *set, int64_t count,
                            int32_t *nearest, double *u) {
  double best = INFINITY;
  int32_t arg = -1;
  for (int64_t k = 0; k < count; k++) {
    if (set[k] == centre) continue;
    double d[3];
    min_image(&pos[3 * centre], &pos[3 * set[k]], box, d);
    const double r = sqrt(sq_dist(d));
    if (r < best) {
      best = r;
      arg = set[k];
      if (u)
        for (int a = 0; a < 3; a++) u[a] = d[a] / r;
    }
  }
  if (nearest) *nearest = arg;
  return best;
}

/* ------------------------------------------------------------------------ */
/* Free energy from a biased trajectory by reweighting (paper, Methods: the  */
/* unbiased probability is the biased average of delta(s - s(R)) e^{beta V}  */
/* over the biased average of e^{beta V}, and F = -(1/beta) log P).  Samples */
/* (s_t, V_t), t = 0..T-1, with s_t of dims <= 2 components; bin i_d =       */
/* floor((s_d - lo_d) / w_d), w_d = (hi_d - lo_d) / nb_d, bin id i_0 +        */
/* nb_0 i_1.  Samples outside the grid count in the denominator only.  The   */
/* weights exp((V_t - V_max)/kBT) share one factor that cancels in P, and    */
/* each sum runs in sample order.  F = -kBT log P per bin; +inf where no     */
/* sample fell.                                                               */
/* ------------------------------------------------------------------------ */
void gmo_fes_reweight(const double *s, const double *V, int64_t T, int dims,
                      const double *lo, const double *hi, const int32_t *nb,
                      double kBT, double *F) {
  int64_t nbins = 1;
  for (int d = 0; d < dims; d++) nbins *= nb[d];
  double vmax = -INFINITY;
  for (int64_t t = 0; t < T; t++)
    if (V[t] > vmax) vmax = V[t];
  double *num = (double *)calloc((size_t)nbins, sizeof(double));
  double den = 0.0;
  for (int64_t t = 0; t < T; t++) {
    const double w = exp((V[t] - vmax) / kBT);
    den += w;
    int64_t bin = 0, stride = 1, inside = 1;
    for (int d = 0; d < dims; d++) {
      const double width = (hi[d] - lo[d]) / nb[d];
      const double x = floor((s[t * dims + d] - lo[d]) / width);
      if (!(x >= 0.0 && x < nb[d])) inside = 0;
      else bin += (int64_t)x * stride;
      stride *= nb[d];
    }
    if (inside) num[bin] += w;
  }
  for (int64_t b = 0; b < nbins; b++)
    F[b] = num[b] > 0.0 ? -kBT * log(num[b] / den) : INFINITY;
  free(num);
}

/* Free energy from the deposited bias itself on the grid of bin centres:
 * F = -V (plain metadynamics) or F = -gamma/(gamma - 1) V (well-tempered,
 * Barducci, Bussi and Parrinello 2008), up to a constant.                   */
void gmo_fes_hills(const double *centres, const double *heights, int64_t K,
                   int dims, const double *sigma, const double *period,
                   double gamma, const double *lo, const double *hi,
                   const int32_t *nb, double *F) {
  const int32_t n1 = dims > 1 ? nb[1] : 1;
  const double scale = gamma > 1.0 ? gamma / (gamma - 1.0) : 1.0;
  for (int32_t i1 = 0; i1 < n1; i1++)
    for (int32_t i0 = 0; i0 < nb[0]; i0++) {
      double g[2];
      g[0] = lo[0] + (i0 + 0.5) * ((hi[0] - lo[0]) / nb[0]);
      if (dims > 1) g[1] = lo[1] + (i1 + 0.5) * ((hi[1] - lo[1]) / nb[1]);
      double v;
      gmo_bias(centres, heights, K, dims, sigma, period, g, &v, NULL);
      F[(int64_t)i1 * nb[0] + i0] = -scale * v;
    }
}
