/*
 * FP64 CPU oracle for the short-range non-bonded force calculation of molecular
 * dynamics (Lennard-Jones 12-6 plus cutoff Coulomb, cell list over the 3x3x3
 * neighbouring cells).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, plain reference that the GPU
 * library is checked against. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it. It shares no code, header, table or
 * constant with the GPU library.
 *
 * What it computes (units: A, e, kcal/mol):
 *   - Eq. 1 (Section 2.1): F_LJ = (A/|r|^14 - B/|r|^8) r, with A = 48 eps s^12 and
 *     B = 24 eps s^6, i.e. A = 12 c12, B = 6 c6 for c12 = 4 eps s^12, c6 = 4 eps s^6.
 *     Mixed-type parameters use Lorentz-Berthelot: s_ij = (s_i + s_j)/2,
 *     eps_ij = sqrt(eps_i eps_j).
 *   - Eq. 2 (Section 2.1): F_C = k q1 q2 / |r|^3 r.
 *   - Cutoff (Section 2.1): a pair interacts only if |r|^2 < rc^2 (strict).
 *   - Reading of r: r = x_i - x_j, so the force on atom i is +f r and a positive
 *     f pushes the two atoms apart.
 *   - Switching (the workload switches from r_switch to r_cut; the paper has none):
 *     the whole pair energy e(u) = c12/u^6 - c6/u^3 + k qi qj / sqrt(u), u = |r|^2,
 *     is multiplied by the smoothstep S(u) = (rc2-u)^2 (rc2+2u-3rs2)/(rc2-rs2)^3 on
 *     (rs2, rc2), S = 1 below rs2; forces are minus the gradient of S(u) e(u).
 *     With the TRUNCATED_COULOMB flag, only the LJ energy is switched and the
 *     Coulomb term is Eq. 2 up to the cutoff.
 *   - Energy: the sum of S(u) e(u) over unique pairs (i < j) within the cutoff.
 *
 * Two independent evaluations of the same sums:
 *   - mdo_forces_bruteforce / mdo_forces_subset: the definition written out, an
 *     O(N^2) minimum-image double loop (valid because every box edge is at least
 *     twice the cutoff, so at most one periodic image lies within the cutoff).
 *   - mdo_forces_celllist: Algorithm 1 (Section 2.1) -- foreach home cell, foreach
 *     of its 27 neighbour cells (periodic images), foreach home atom, foreach atom
 *     of the neighbour cell, test the cutoff and accumulate the force on the home
 *     atom. Each pair is visited from both of its atoms, as in Algorithm 1.
 *     Cells are flat arrays filled by a stable counting sort (Section 2.2, second
 *     transformation: linked-list cells become arrays).
 *
 * Cell grid (cell edge at least the cutoff, Section 2.1 and the 27-cell stencil
 * of Fig. 2): n_d = floor(L_d / rc); if L_d/n_d - rc < 1e-3 A the grid takes
 * n_d - 1 cells so that rounding at a cell face can never hide a pair; fewer than
 * 2 cells on an axis (L_d < 2 rc) is rejected.
 *
 * Beyond the cutoff (Section 2.1 hands the long-range Coulomb force to an O(N)
 * approximation on the CPU), read as Ewald summation: with MDO_FLAG_EWALD the Coulomb
 * term inside the cutoff is the real-space part k qi qj erfc(alpha r)/r (only the LJ
 * energy switched), and mdo_ewald_recip sums the reciprocal-space part, the self term
 * and the neutralising background plainly over wave vectors.
 *
 * Canonicalisation: positions in [-L, 2L) are wrapped into [0, L] by one add or
 * subtract of L in the precision of the input (float32 inputs are wrapped in
 * float32, then promoted exactly to double). NaN or positions outside [-L, 2L)
 * are reported through status bits.
 *
 * Build: gcc -O2 -std=c11 -fopenmp -ffp-contract=off -fPIC -shared.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MDO_OK 0
#define MDO_ERR_ARG (-1)
#define MDO_ERR_BOX (-2)
#define MDO_ERR_CAPACITY (-6)
#define MDO_ERR_NOMEM (-7)

#define MDO_FLAG_TRUNCATED_COULOMB (1u << 1)
#define MDO_FLAG_EWALD (1u << 7)
#define MDO_PI 3.14159265358979323846

#define MDO_STATUS_NAN (1u << 0)
#define MDO_STATUS_OUT_OF_BOX (1u << 1)
#define MDO_STATUS_BAD_TYPE (1u << 2)

typedef struct {
  double box[3];
  double r_cut;
  double r_switch;
  double coulomb_k;
  int32_t n_types;
  const double* sigma;
  const double* epsilon;
  uint32_t flags;
  double ewald_alpha; /* 1/A, with MDO_FLAG_EWALD */
} mdo_params;

/* Per-call constants: the mixed LJ table and the switching constants. */
typedef struct {
  int nt;
  double* c12; /* [nt*nt] 4 eps_ij s_ij^12 */
  double* c6;  /* [nt*nt] 4 eps_ij s_ij^6  */
  double rc2, rs2, k;
  int switching;
  int truncated_coulomb;
  int ewald;
  double alpha;
  double L[3];
} ctx_t;

static int ctx_init(ctx_t* c, const mdo_params* p) {
  if (!p || p->n_types < 1 || !p->sigma || !p->epsilon) return MDO_ERR_ARG;
  if (!(p->r_cut > 0) || !(p->r_switch > 0) || p->r_switch > p->r_cut) return MDO_ERR_ARG;
  for (int d = 0; d < 3; ++d) {
    if (!(p->box[d] >= 2.0 * p->r_cut)) return MDO_ERR_BOX;
    c->L[d] = p->box[d];
  }
  int nt = p->n_types;
  c->nt = nt;
  c->c12 = (double*)malloc(sizeof(double) * nt * nt);
  c->c6 = (double*)malloc(sizeof(double) * nt * nt);
  if (!c->c12 || !c->c6) {
    free(c->c12);
    free(c->c6);
    return MDO_ERR_NOMEM;
  }
  for (int a = 0; a < nt; ++a)
    for (int b = 0; b < nt; ++b) {
      double s = 0.5 * (p->sigma[a] + p->sigma[b]);
      double e = sqrt(p->epsilon[a] * p->epsilon[b]);
      double s2 = s * s, s6 = s2 * s2 * s2;
      c->c6[a * nt + b] = 4.0 * e * s6;
      c->c12[a * nt + b] = 4.0 * e * s6 * s6;
    }
  c->rc2 = p->r_cut * p->r_cut;
  c->rs2 = p->r_switch * p->r_switch;
  c->k = p->coulomb_k;
  c->switching = p->r_switch < p->r_cut;
  c->truncated_coulomb = (p->flags & MDO_FLAG_TRUNCATED_COULOMB) != 0;
  c->ewald = (p->flags & MDO_FLAG_EWALD) != 0;
  c->alpha = p->ewald_alpha;
  if (c->ewald && !(c->alpha > 0)) {
    free(c->c12);
    free(c->c6);
    return MDO_ERR_ARG;
  }
  return MDO_OK;
}

static void ctx_free(ctx_t* c) {
  free(c->c12);
  free(c->c6);
}

/* Switching function S(u) and its derivative dS/du on u = r^2. */
static void switch_fn(const ctx_t* c, double u, double* S, double* dS) {
  if (!c->switching || u <= c->rs2) {
    *S = 1.0;
    *dS = 0.0;
    return;
  }
  double w = c->rc2 - c->rs2;
  double w3 = w * w * w;
  double a = c->rc2 - u;
  *S = a * a * (c->rc2 + 2.0 * u - 3.0 * c->rs2) / w3;
  *dS = 6.0 * a * (c->rs2 - u) / w3;
}

/*
 * One pair at squared distance u (< rc2). Returns the scalar f with
 * F_i = f * (x_i - x_j) and F_j = -F_i; stores the pair energy in *e.
 * Eq. 1 and Eq. 2 give, for the unswitched terms,
 *   f_LJ = 12 c12 / u^7 - 6 c6 / u^4,   f_C = k qi qj / u^(3/2),
 * and the switched force is -2 d(S e)/du = S (f_LJ + f_C) - 2 S' e.
 */
static double pair_fe(const ctx_t* c, int ti, int tj, double qi, double qj, double u,
                      double* e) {
  double c12 = c->c12[ti * c->nt + tj];
  double c6 = c->c6[ti * c->nt + tj];
  double inv_u = 1.0 / u;
  double inv_u3 = inv_u * inv_u * inv_u;
  double e_lj = c12 * inv_u3 * inv_u3 - c6 * inv_u3;
  double f_lj = (12.0 * c12 * inv_u3 * inv_u3 - 6.0 * c6 * inv_u3) * inv_u;
  double r = sqrt(u);
  double e_c = c->k * qi * qj / r;
  double f_c = e_c * inv_u;
  double S, dS;
  switch_fn(c, u, &S, &dS);
  if (c->ewald) {
    /* Ewald real-space term (the Coulomb energy split as erfc + erf, the erf part summed
     * in reciprocal space): e = k qi qj erfc(alpha r) / r, and
     * f = -(1/r) de/dr = k qi qj (erfc(alpha r)/r + 2 alpha/sqrt(pi) exp(-alpha^2 r^2)) / r^2;
     * only the LJ energy is switched */
    const double ar = c->alpha * r;
    e_c = c->k * qi * qj * erfc(ar) / r;
    f_c = c->k * qi * qj * (erfc(ar) / r + 2.0 * c->alpha / sqrt(MDO_PI) * exp(-ar * ar)) * inv_u;
    *e = S * e_lj + e_c;
    return S * f_lj - 2.0 * dS * e_lj + f_c;
  }
  if (c->truncated_coulomb) {
    *e = S * e_lj + e_c;
    return S * f_lj - 2.0 * dS * e_lj + f_c;
  }
  *e = S * (e_lj + e_c);
  return S * (f_lj + f_c) - 2.0 * dS * (e_lj + e_c);
}

/* ---------------------------------------------------------------- grid ---- */

int mdo_grid(const mdo_params* p, int32_t dims[3]) {
  if (!p || !(p->r_cut > 0)) return MDO_ERR_ARG;
  for (int d = 0; d < 3; ++d) {
    double L = p->box[d];
    if (!(L >= 2.0 * p->r_cut)) return MDO_ERR_BOX;
    int n = (int)floor(L / p->r_cut);
    if (L / n - p->r_cut < 1e-3) n -= 1;
    if (n < 2) return MDO_ERR_BOX;
    dims[d] = n;
  }
  return MDO_OK;
}

static int cell_coord(double x, double L, int n) {
  int c = (int)floor(x * (double)n / L);
  if (c < 0) c = 0;
  if (c > n - 1) c = n - 1;
  return c;
}

/* Cell index (iz*ny + iy)*nx + ix of every atom; positions must be canonical. */
int mdo_bin(const mdo_params* p, int64_t n, const double* pos, int32_t* cell_out,
            int32_t dims_out[3]) {
  int32_t dims[3];
  int rc = mdo_grid(p, dims);
  if (rc) return rc;
  for (int64_t i = 0; i < n; ++i) {
    int ix = cell_coord(pos[3 * i + 0], p->box[0], dims[0]);
    int iy = cell_coord(pos[3 * i + 1], p->box[1], dims[1]);
    int iz = cell_coord(pos[3 * i + 2], p->box[2], dims[2]);
    cell_out[i] = (iz * dims[1] + iy) * dims[0] + ix;
  }
  if (dims_out) memcpy(dims_out, dims, sizeof(dims));
  return MDO_OK;
}

/* ------------------------------------------------------- canonicalise ---- */

int mdo_canonicalize_f32(int64_t n, const float* pos, const double box[3], double* out,
                         uint32_t* status) {
  uint32_t st = 0;
  for (int d = 0; d < 3; ++d) {
    float L = (float)box[d];
    for (int64_t i = 0; i < n; ++i) {
      float x = pos[3 * i + d];
      if (isnan(x)) {
        st |= MDO_STATUS_NAN;
      } else if (x < -L || x >= 2.0f * L) {
        st |= MDO_STATUS_OUT_OF_BOX;
      } else if (x < 0.0f) {
        x = x + L; /* one float32 rounding */
      } else if (x >= L) {
        x = x - L; /* exact (Sterbenz) */
      }
      out[3 * i + d] = (double)x;
    }
  }
  if (status) *status = st;
  return MDO_OK;
}

int mdo_canonicalize_f64(int64_t n, const double* pos, const double box[3], double* out,
                         uint32_t* status) {
  uint32_t st = 0;
  for (int d = 0; d < 3; ++d) {
    double L = box[d];
    for (int64_t i = 0; i < n; ++i) {
      double x = pos[3 * i + d];
      if (isnan(x)) {
        st |= MDO_STATUS_NAN;
      } else if (x < -L || x >= 2.0 * L) {
        st |= MDO_STATUS_OUT_OF_BOX;
      } else if (x < 0.0) {
        x = x + L;
      } else if (x >= L) {
        x = x - L;
      }
      out[3 * i + d] = x;
    }
  }
  if (status) *status = st;
  return MDO_OK;
}

static int check_types(const mdo_params* p, int64_t n, const int32_t* type) {
  for (int64_t i = 0; i < n; ++i)
    if (type[i] < 0 || type[i] >= p->n_types) return MDO_ERR_ARG;
  return MDO_OK;
}

/* ------------------------------------------------------ pair function ---- */

/* Scalar pair terms for one pair of types and charges at squared distance u.
 * Writes 0 to both outputs when u >= rc^2. */
int mdo_pair_terms(const mdo_params* p, int32_t ti, int32_t tj, double qi, double qj,
                   double u, double* e_out, double* f_out) {
  ctx_t c;
  mdo_params q = *p;
  for (int d = 0; d < 3; ++d) q.box[d] = 2.0 * p->r_cut; /* box irrelevant here */
  int rc = ctx_init(&c, &q);
  if (rc) return rc;
  if (ti < 0 || tj < 0 || ti >= c.nt || tj >= c.nt) {
    ctx_free(&c);
    return MDO_ERR_ARG;
  }
  double e = 0.0, f = 0.0;
  if (u < c.rc2) f = pair_fe(&c, ti, tj, qi, qj, u, &e);
  *e_out = e;
  *f_out = f;
  ctx_free(&c);
  return MDO_OK;
}

/* Minimum-image displacement r = x_i - x_j (exact for float32-origin inputs). */
static inline void min_image(const ctx_t* c, const double* xi, const double* xj,
                             double r[3]) {
  for (int d = 0; d < 3; ++d) {
    double v = xi[d] - xj[d];
    v -= c->L[d] * nearbyint(v / c->L[d]);
    r[d] = v;
  }
}

static inline double norm2(const double r[3]) {
  return r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
}

/* --------------------------------------------------- O(N^2) definition ---- */

/*
 * Forces on the atoms listed in idx (or on all atoms if idx is NULL), each summed
 * over every other atom by minimum image. Energy and pair count are over unique
 * pairs and only produced when idx is NULL. Optional per-atom outputs: the sum of
 * pair-force magnitudes |f_ij r_ij| (the conditioning of the sum) and the number
 * of partners within the cutoff.
 */
static int forces_direct(const mdo_params* p, int64_t n, const double* pos,
                         const int32_t* type, const double* q, int64_t n_idx,
                         const int64_t* idx, double* force, double* energy,
                         int64_t* n_pairs, double* abs_sum, int64_t* count,
                         int n_threads) {
  ctx_t c;
  int rc = ctx_init(&c, p);
  if (rc) return rc;
  if (check_types(p, n, type)) {
    ctx_free(&c);
    return MDO_ERR_ARG;
  }
  int64_t m = idx ? n_idx : n;
  double* e_part = (double*)calloc((size_t)(m > 0 ? m : 1), sizeof(double));
  int64_t* p_part = (int64_t*)calloc((size_t)(m > 0 ? m : 1), sizeof(int64_t));
  if (!e_part || !p_part) {
    free(e_part);
    free(p_part);
    ctx_free(&c);
    return MDO_ERR_NOMEM;
  }
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
  for (int64_t a = 0; a < m; ++a) {
    int64_t i = idx ? idx[a] : a;
    double F[3] = {0, 0, 0}, asum = 0.0, esum = 0.0;
    int64_t cnt = 0, pairs = 0;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double r[3];
      min_image(&c, pos + 3 * i, pos + 3 * j, r);
      double u = norm2(r);
      if (!(u < c.rc2)) continue;
      double e;
      double f = pair_fe(&c, type[i], type[j], q[i], q[j], u, &e);
      for (int d = 0; d < 3; ++d) F[d] += f * r[d];
      asum += fabs(f) * sqrt(u);
      cnt += 1;
      if (j > i) {
        esum += e;
        pairs += 1;
      }
    }
    for (int d = 0; d < 3; ++d) force[3 * a + d] = F[d];
    if (abs_sum) abs_sum[a] = asum;
    if (count) count[a] = cnt;
    e_part[a] = esum;
    p_part[a] = pairs;
  }
  if (!idx) {
    double E = 0.0;
    int64_t P = 0;
    for (int64_t a = 0; a < m; ++a) {
      E += e_part[a];
      P += p_part[a];
    }
    if (energy) *energy = E;
    if (n_pairs) *n_pairs = P;
  }
  free(e_part);
  free(p_part);
  ctx_free(&c);
  return MDO_OK;
}

int mdo_forces_bruteforce(const mdo_params* p, int64_t n, const double* pos,
                          const int32_t* type, const double* q, double* force,
                          double* energy, int64_t* n_pairs, double* abs_sum,
                          int64_t* count, int n_threads) {
  if (!p || n < 0 || (n > 0 && (!pos || !type || !q || !force))) return MDO_ERR_ARG;
  return forces_direct(p, n, pos, type, q, 0, NULL, force, energy, n_pairs, abs_sum,
                       count, n_threads);
}

int mdo_forces_subset(const mdo_params* p, int64_t n, const double* pos,
                      const int32_t* type, const double* q, int64_t n_idx,
                      const int64_t* idx, double* force, double* abs_sum, int64_t* count,
                      int n_threads) {
  if (!p || n < 0 || n_idx < 0 || (n_idx > 0 && !idx) || !force) return MDO_ERR_ARG;
  for (int64_t a = 0; a < n_idx; ++a)
    if (idx[a] < 0 || idx[a] >= n) return MDO_ERR_ARG;
  return forces_direct(p, n, pos, type, q, n_idx, idx, force, NULL, NULL, abs_sum, count,
                       n_threads);
}

/* ------------------------------------------------- cell list (Alg. 1) ---- */

typedef struct {
  int32_t dims[3];
  int64_t n_cells;
  int64_t* start; /* [n_cells+1] */
  int64_t* atoms; /* [n] original indices, cell-major, stable within a cell */
} cells_t;

static int cells_build(const mdo_params* p, int64_t n, const double* pos, cells_t* cl) {
  int rc = mdo_grid(p, cl->dims);
  if (rc) return rc;
  cl->n_cells = (int64_t)cl->dims[0] * cl->dims[1] * cl->dims[2];
  cl->start = (int64_t*)calloc((size_t)cl->n_cells + 1, sizeof(int64_t));
  cl->atoms = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int32_t* cell = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  if (!cl->start || !cl->atoms || !cell) {
    free(cl->start);
    free(cl->atoms);
    free(cell);
    return MDO_ERR_NOMEM;
  }
  mdo_bin(p, n, pos, cell, NULL);
  /* counting sort: count, exclusive scan, stable scatter */
  for (int64_t i = 0; i < n; ++i) cl->start[cell[i] + 1] += 1;
  for (int64_t c = 0; c < cl->n_cells; ++c) cl->start[c + 1] += cl->start[c];
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)cl->n_cells);
  if (!fill) {
    free(cl->start);
    free(cl->atoms);
    free(cell);
    return MDO_ERR_NOMEM;
  }
  memcpy(fill, cl->start, sizeof(int64_t) * (size_t)cl->n_cells);
  for (int64_t i = 0; i < n; ++i) cl->atoms[fill[cell[i]]++] = i;
  free(fill);
  free(cell);
  return MDO_OK;
}

static void cells_free(cells_t* cl) {
  free(cl->start);
  free(cl->atoms);
}

/* Visits every (home atom, neighbour atom image) pair within the cutoff, in the
 * loop order of Algorithm 1, calling the visitor with the displacement
 * r = x_home - x_neighbour_image. */
typedef void (*visit_fn)(void* ud, int64_t i, int64_t j, const double r[3], double u);

static void celllist_home_cell(const ctx_t* c, const cells_t* cl, const double* pos,
                               int64_t hc, visit_fn fn, void* ud) {
  int nx = cl->dims[0], ny = cl->dims[1], nz = cl->dims[2];
  int hx = (int)(hc % nx), hy = (int)((hc / nx) % ny), hz = (int)(hc / ((int64_t)nx * ny));
  for (int oz = -1; oz <= 1; ++oz)
    for (int oy = -1; oy <= 1; ++oy)
      for (int ox = -1; ox <= 1; ++ox) {
        /* neighbour cell and the periodic shift of its image */
        int b[3] = {hx + ox, hy + oy, hz + oz};
        int dim[3] = {nx, ny, nz};
        double shift[3];
        for (int d = 0; d < 3; ++d) {
          shift[d] = 0.0;
          if (b[d] < 0) {
            b[d] += dim[d];
            shift[d] = -c->L[d];
          } else if (b[d] >= dim[d]) {
            b[d] -= dim[d];
            shift[d] = c->L[d];
          }
        }
        int64_t nc = ((int64_t)b[2] * ny + b[1]) * nx + b[0];
        for (int64_t a = cl->start[hc]; a < cl->start[hc + 1]; ++a) {
          int64_t i = cl->atoms[a];
          for (int64_t bb = cl->start[nc]; bb < cl->start[nc + 1]; ++bb) {
            int64_t j = cl->atoms[bb];
            if (ox == 0 && oy == 0 && oz == 0 && j == i) continue;
            double r[3];
            for (int d = 0; d < 3; ++d) r[d] = pos[3 * i + d] - (pos[3 * j + d] + shift[d]);
            double u = norm2(r);
            if (u < c->rc2) fn(ud, i, j, r, u);
          }
        }
      }
}

typedef struct {
  const ctx_t* c;
  const int32_t* type;
  const double* q;
  double* force;
  double* abs_sum;
  int64_t* count;
  double e;
  int64_t pairs;
} force_ud;

static void visit_force(void* vud, int64_t i, int64_t j, const double r[3], double u) {
  force_ud* ud = (force_ud*)vud;
  double e;
  double f = pair_fe(ud->c, ud->type[i], ud->type[j], ud->q[i], ud->q[j], u, &e);
  for (int d = 0; d < 3; ++d) ud->force[3 * i + d] += f * r[d];
  if (ud->abs_sum) ud->abs_sum[i] += fabs(f) * sqrt(u);
  if (ud->count) ud->count[i] += 1;
  if (i < j) {
    ud->e += e;
    ud->pairs += 1;
  }
}

int mdo_forces_celllist(const mdo_params* p, int64_t n, const double* pos,
                        const int32_t* type, const double* q, double* force,
                        double* energy, int64_t* n_pairs, double* abs_sum, int64_t* count,
                        int n_threads) {
  if (!p || n < 0 || (n > 0 && (!pos || !type || !q || !force))) return MDO_ERR_ARG;
  ctx_t c;
  int rc = ctx_init(&c, p);
  if (rc) return rc;
  if (check_types(p, n, type)) {
    ctx_free(&c);
    return MDO_ERR_ARG;
  }
  cells_t cl;
  rc = cells_build(p, n, pos, &cl);
  if (rc) {
    ctx_free(&c);
    return rc;
  }
  memset(force, 0, sizeof(double) * 3 * (size_t)n);
  if (abs_sum) memset(abs_sum, 0, sizeof(double) * (size_t)n);
  if (count) memset(count, 0, sizeof(int64_t) * (size_t)n);
  double* e_cell = (double*)calloc((size_t)cl.n_cells, sizeof(double));
  int64_t* p_cell = (int64_t*)calloc((size_t)cl.n_cells, sizeof(int64_t));
  if (!e_cell || !p_cell) {
    free(e_cell);
    free(p_cell);
    cells_free(&cl);
    ctx_free(&c);
    return MDO_ERR_NOMEM;
  }
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int64_t hc = 0; hc < cl.n_cells; ++hc) {
    /* each home cell writes only the forces of its own atoms */
    force_ud ud = {&c, type, q, force, abs_sum, count, 0.0, 0};
    celllist_home_cell(&c, &cl, pos, hc, visit_force, &ud);
    e_cell[hc] = ud.e;
    p_cell[hc] = ud.pairs;
  }
  double E = 0.0;
  int64_t P = 0;
  for (int64_t hc = 0; hc < cl.n_cells; ++hc) {
    E += e_cell[hc];
    P += p_cell[hc];
  }
  if (energy) *energy = E;
  if (n_pairs) *n_pairs = P;
  free(e_cell);
  free(p_cell);
  cells_free(&cl);
  ctx_free(&c);
  return MDO_OK;
}

/* ----------------------------------------------------------- pair sets ---- */

static int cmp_pair(const void* a, const void* b) {
  const int32_t* x = (const int32_t*)a;
  const int32_t* y = (const int32_t*)b;
  if (x[0] != y[0]) return x[0] < y[0] ? -1 : 1;
  if (x[1] != y[1]) return x[1] < y[1] ? -1 : 1;
  return 0;
}

/* Unique pairs (i < j) within the cutoff by the O(N^2) definition, in
 * lexicographic order. Writes at most cap pairs; *n_pairs gets the true count. */
int mdo_pairs_bruteforce(const mdo_params* p, int64_t n, const double* pos, int64_t cap,
                         int64_t* n_pairs, int32_t* pairs) {
  ctx_t c;
  mdo_params pp = *p;
  double one = 1.0, zero = 0.0;
  pp.n_types = 1;
  pp.sigma = &one;
  pp.epsilon = &zero;
  int rc = ctx_init(&c, &pp);
  if (rc) return rc;
  int64_t k = 0;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = i + 1; j < n; ++j) {
      double r[3];
      min_image(&c, pos + 3 * i, pos + 3 * j, r);
      if (norm2(r) < c.rc2) {
        if (k < cap) {
          pairs[2 * k] = (int32_t)i;
          pairs[2 * k + 1] = (int32_t)j;
        }
        ++k;
      }
    }
  *n_pairs = k;
  ctx_free(&c);
  return k > cap ? MDO_ERR_CAPACITY : MDO_OK;
}

typedef struct {
  int64_t k, cap;
  int32_t* pairs;
} pairs_ud;

static void visit_pair(void* vud, int64_t i, int64_t j, const double r[3], double u) {
  (void)r;
  (void)u;
  pairs_ud* ud = (pairs_ud*)vud;
  if (i >= j) return;
  if (ud->k < ud->cap) {
    ud->pairs[2 * ud->k] = (int32_t)i;
    ud->pairs[2 * ud->k + 1] = (int32_t)j;
  }
  ud->k += 1;
}

/* Unique pairs found by the cell list (Algorithm 1 traversal), sorted. */
int mdo_pairs_celllist(const mdo_params* p, int64_t n, const double* pos, int64_t cap,
                       int64_t* n_pairs, int32_t* pairs) {
  ctx_t c;
  mdo_params pp = *p;
  double one = 1.0, zero = 0.0;
  pp.n_types = 1;
  pp.sigma = &one;
  pp.epsilon = &zero;
  int rc = ctx_init(&c, &pp);
  if (rc) return rc;
  cells_t cl;
  rc = cells_build(&pp, n, pos, &cl);
  if (rc) {
    ctx_free(&c);
    return rc;
  }
  pairs_ud ud = {0, cap, pairs};
  for (int64_t hc = 0; hc < cl.n_cells; ++hc) celllist_home_cell(&c, &cl, pos, hc, visit_pair, &ud);
  *n_pairs = ud.k;
  if (ud.k <= cap) qsort(pairs, (size_t)ud.k, 2 * sizeof(int32_t), cmp_pair);
  cells_free(&cl);
  ctx_free(&c);
  return ud.k > cap ? MDO_ERR_CAPACITY : MDO_OK;
}

/* Per-atom count of partners whose squared distance lies within band of rc^2
 * (|u - rc^2| <= band): the pairs whose inclusion may differ between a float32
 * and a float64 evaluation of the cutoff test. Returns the number of such pairs. */
int mdo_band_atoms(const mdo_params* p, int64_t n, const double* pos, double band,
                   int64_t* n_band_pairs, int64_t* per_atom, int n_threads) {
  ctx_t c;
  mdo_params pp = *p;
  double one = 1.0, zero = 0.0;
  pp.n_types = 1;
  pp.sigma = &one;
  pp.epsilon = &zero;
  int rc = ctx_init(&c, &pp);
  if (rc) return rc;
  cells_t cl;
  rc = cells_build(&pp, n, pos, &cl);
  if (rc) {
    ctx_free(&c);
    return rc;
  }
  memset(per_atom, 0, sizeof(int64_t) * (size_t)n);
  int64_t total = 0;
  int nx = cl.dims[0], ny = cl.dims[1], nz = cl.dims[2];
  /* plain full-shell traversal with a widened test */
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : total)
#endif
  for (int64_t hc = 0; hc < cl.n_cells; ++hc) {
    int hx = (int)(hc % nx), hy = (int)((hc / nx) % ny), hz = (int)(hc / ((int64_t)nx * ny));
    for (int oz = -1; oz <= 1; ++oz)
      for (int oy = -1; oy <= 1; ++oy)
        for (int ox = -1; ox <= 1; ++ox) {
          int b[3] = {hx + ox, hy + oy, hz + oz};
          int dim[3] = {nx, ny, nz};
          double shift[3];
          for (int d = 0; d < 3; ++d) {
            shift[d] = 0.0;
            if (b[d] < 0) {
              b[d] += dim[d];
              shift[d] = -c.L[d];
            } else if (b[d] >= dim[d]) {
              b[d] -= dim[d];
              shift[d] = c.L[d];
            }
          }
          int64_t nc = ((int64_t)b[2] * ny + b[1]) * nx + b[0];
          for (int64_t a = cl.start[hc]; a < cl.start[hc + 1]; ++a) {
            int64_t i = cl.atoms[a];
            for (int64_t bb = cl.start[nc]; bb < cl.start[nc + 1]; ++bb) {
              int64_t j = cl.atoms[bb];
              if (ox == 0 && oy == 0 && oz == 0 && j == i) continue;
              double r[3];
              for (int d = 0; d < 3; ++d) r[d] = pos[3 * i + d] - (pos[3 * j + d] + shift[d]);
              if (fabs(norm2(r) - c.rc2) <= band) {
                per_atom[i] += 1;
                if (i < j) total += 1;
              }
            }
          }
        }
  }
  *n_band_pairs = total;
  cells_free(&cl);
  ctx_free(&c);
  return MDO_OK;
}

/* --------------------------------------------- Ewald reciprocal space ---- */

/*
 * The Coulomb interaction beyond the cutoff (Section 2.1 leaves it to an O(N)
 * approximation outside the short-range kernel). Read here as Ewald summation for the
 * periodic box: with the real-space erfc term inside the cutoff (MDO_FLAG_EWALD), the
 * rest of the Coulomb energy is
 *   E_recip = k/(2V) sum_{kv != 0} (4 pi / |kv|^2) exp(-|kv|^2 / (4 alpha^2)) |S(kv)|^2,
 *   S(kv)   = sum_j q_j exp(i kv . r_j),   kv = 2 pi (mx/Lx, my/Ly, mz/Lz),
 *   E_self  = -k alpha / sqrt(pi) sum_j q_j^2,
 *   E_bg    = -k pi Q^2 / (2 V alpha^2)   (neutralising background for net charge Q),
 * summed here over every kv with |m_d| <= kmax_d, written out plainly (no symmetry,
 * no tables), and
 *   F_i = -dE_recip/dr_i = (4 pi k q_i / V) sum_kv (kv / |kv|^2) exp(-|kv|^2/(4 alpha^2))
 *         Im(conj(S(kv)) exp(i kv . r_i)).
 */
int mdo_ewald_recip(const mdo_params* p, int64_t n, const double* pos, const double* q,
                    const int32_t kmax[3], double* force, double* e_recip, double* e_self,
                    double* e_bg, int n_threads) {
  if (!p || n < 0 || (n > 0 && (!pos || !q)) || !kmax || !(p->ewald_alpha > 0)) return MDO_ERR_ARG;
  for (int d = 0; d < 3; ++d)
    if (kmax[d] < 0 || !(p->box[d] > 0)) return MDO_ERR_ARG;
  const double a = p->ewald_alpha, k = p->coulomb_k;
  const double V = p->box[0] * p->box[1] * p->box[2];
  const int64_t nx = 2 * kmax[0] + 1, ny = 2 * kmax[1] + 1, nz = 2 * kmax[2] + 1;
  const int64_t nk = nx * ny * nz;
  double* sre = (double*)calloc((size_t)nk, sizeof(double));
  double* sim = (double*)calloc((size_t)nk, sizeof(double));
  double* ek = (double*)calloc((size_t)nk, sizeof(double));
  if (!sre || !sim || !ek) {
    free(sre);
    free(sim);
    free(ek);
    return MDO_ERR_NOMEM;
  }
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(static)
#endif
  for (int64_t t = 0; t < nk; ++t) {
    const int mx = (int)(t / (ny * nz)) - kmax[0];
    const int my = (int)((t / nz) % ny) - kmax[1];
    const int mz = (int)(t % nz) - kmax[2];
    if (mx == 0 && my == 0 && mz == 0) continue;
    const double kv[3] = {2.0 * MDO_PI * mx / p->box[0], 2.0 * MDO_PI * my / p->box[1],
                          2.0 * MDO_PI * mz / p->box[2]};
    const double k2 = kv[0] * kv[0] + kv[1] * kv[1] + kv[2] * kv[2];
    double re = 0.0, im = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      const double th = kv[0] * pos[3 * j] + kv[1] * pos[3 * j + 1] + kv[2] * pos[3 * j + 2];
      re += q[j] * cos(th);
      im += q[j] * sin(th);
    }
    sre[t] = re;
    sim[t] = im;
    ek[t] = k / (2.0 * V) * (4.0 * MDO_PI / k2) * exp(-k2 / (4.0 * a * a)) * (re * re + im * im);
  }
  double E = 0.0;
  for (int64_t t = 0; t < nk; ++t) E += ek[t];
  if (force) {
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int64_t i = 0; i < n; ++i) {
      double F[3] = {0.0, 0.0, 0.0};
      for (int64_t t = 0; t < nk; ++t) {
        const int mx = (int)(t / (ny * nz)) - kmax[0];
        const int my = (int)((t / nz) % ny) - kmax[1];
        const int mz = (int)(t % nz) - kmax[2];
        if (mx == 0 && my == 0 && mz == 0) continue;
        const double kv[3] = {2.0 * MDO_PI * mx / p->box[0], 2.0 * MDO_PI * my / p->box[1],
                              2.0 * MDO_PI * mz / p->box[2]};
        const double k2 = kv[0] * kv[0] + kv[1] * kv[1] + kv[2] * kv[2];
        const double th = kv[0] * pos[3 * i] + kv[1] * pos[3 * i + 1] + kv[2] * pos[3 * i + 2];
        /* Im(conj(S) e^{i th}) = S_re sin(th) - S_im cos(th) */
        const double w = exp(-k2 / (4.0 * a * a)) / k2 * (sre[t] * sin(th) - sim[t] * cos(th));
        for (int d = 0; d < 3; ++d) F[d] += kv[d] * w;
      }
      for (int d = 0; d < 3; ++d) force[3 * i + d] = 4.0 * MDO_PI * k * q[i] / V * F[d];
    }
  }
  double q2 = 0.0, Q = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    q2 += q[j] * q[j];
    Q += q[j];
  }
  if (e_recip) *e_recip = E;
  if (e_self) *e_self = -k * a / sqrt(MDO_PI) * q2;
  if (e_bg) *e_bg = -k * MDO_PI * Q * Q / (2.0 * V * a * a);
  free(sre);
  free(sim);
  free(ek);
  return MDO_OK;
}
