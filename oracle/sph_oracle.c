/*
 * FP64 oracle of the WCSPH / k-epsilon RANS step with improved bidirectional
 * open-boundary buffers (F. Wang, X. Hu, arXiv 2510.25702).
 *
 * TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU-baseline timing).  It
 * shares no code with the HIP library.  Built with -O2 -ffp-contract=off so
 * that every predicate (neighbour cut-off, buffer boxes, cell index) is
 * evaluated as written, without fused multiply-adds.
 *
 * Conventions (readings of the paper, listed in the design notes):
 *  - r_ij = x_i - x_j, r = |r_ij|; grad W_ij = (dW/dr)(r) r_ij / r is the
 *    gradient with respect to x_i (this is what makes the correction matrix
 *    of Sec. 2.2 positive definite);
 *  - the Riemann axis e_ij of the intermediate velocity and of the ARD
 *    limiter points from i to j, e_ij = -r_ij / r (dissipative sign);
 *  - V_j = m_j / rho_j, m = rho0 dp^dim; wall dummy particles have V = dp^dim,
 *    zero velocity, p_w = p_i, rho_w = rho_i and B_w = B_i;
 *  - kernel: Wendland C2 with cut-off 2h.
 */
#include "sph_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define KIND(t) ((int)((t) & 3u))
#define BID(t) ((int)(((t) >> 8) & 0xFFu))
#define MAXNB 4096
#define PI 3.14159265358979323846

static int g_threads = 1;
void ora_set_threads(int n) { g_threads = n > 0 ? n : 1; }
int ora_get_threads(void) { return g_threads; }

/* ------------------------------------------------------------------------ */
/* Counter-based random numbers: SplitMix64 (Steele, Lea & Flood 2014).      */
/* u = 2 * (z >> 11) * 2^-53 - 1 with                                        */
/* z = mix(mix(mix(seed) ^ pid) ^ ((step << 2) | comp)).                     */
/* ------------------------------------------------------------------------ */
uint64_t ora_splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double ora_uniform(uint64_t seed, uint32_t pid, int64_t step, uint32_t comp) {
  uint64_t z = ora_splitmix64(seed);
  z = ora_splitmix64(z ^ (uint64_t)pid);
  z = ora_splitmix64(z ^ (((uint64_t)step << 2) | (uint64_t)comp));
  return (double)(z >> 11) * 0x1.0p-53 * 2.0 - 1.0;
}

/* ------------------------------------------------------------------------ */
/* Kernel W(r, h), Sec. 2.2 (h = 1.3 dp); Wendland C2 with cut-off 2h.       */
/* ------------------------------------------------------------------------ */
static double kernel_alpha(int dim, double h) {
  return dim == 2 ? 7.0 / (4.0 * PI * h * h) : 21.0 / (16.0 * PI * h * h * h);
}

double ora_kernel_W(double r, double h, int dim) {
  double q = r / h;
  if (q >= 2.0) return 0.0;
  double t = 1.0 - 0.5 * q;
  return kernel_alpha(dim, h) * t * t * t * t * (2.0 * q + 1.0);
}

double ora_kernel_dW(double r, double h, int dim) {
  double q = r / h;
  if (q >= 2.0) return 0.0;
  double t = 1.0 - 0.5 * q;
  return kernel_alpha(dim, h) * (-5.0 * q) * t * t * t / h;
}

/* (dW/dr) / r, finite at r = 0 */
static double kernel_dW_over_r(double r, double h, int dim) {
  double q = r / h;
  if (q >= 2.0) return 0.0;
  double t = 1.0 - 0.5 * q;
  return kernel_alpha(dim, h) * (-5.0) * t * t * t / (h * h);
}

/* ------------------------------------------------------------------------ */
/* Cell linked list (Sec. 2.4.1): head/next lists over a uniform grid.       */
/* ------------------------------------------------------------------------ */
typedef struct {
  int dim;
  double lo[3], cs;
  int64_t nc[3], ncell;
  int64_t *head, *next;
} grid_t;

static int64_t cell_coord(double x, double lo, double cs) {
  return (int64_t)floor((x - lo) / cs);
}

static void grid_dims(const ora_params* P, int64_t nc[3]) {
  for (int k = 0; k < 3; ++k)
    nc[k] = (k < P->dim) ? (int64_t)ceil((P->hi[k] - P->lo[k]) / P->cell_size) : 1;
}

static void grid_free(grid_t* g) {
  free(g->head);
  free(g->next);
  g->head = g->next = NULL;
}

/* Returns ORA_E_NUMERIC if a particle is outside the interior of the grid. */
static int grid_build(grid_t* g, const ora_params* P, int64_t n, const double* x) {
  g->dim = P->dim;
  g->cs = P->cell_size;
  for (int k = 0; k < 3; ++k) g->lo[k] = P->lo[k];
  grid_dims(P, g->nc);
  g->ncell = g->nc[0] * g->nc[1] * g->nc[2];
  g->head = (int64_t*)malloc(sizeof(int64_t) * (size_t)g->ncell);
  g->next = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  for (int64_t c = 0; c < g->ncell; ++c) g->head[c] = -1;
  int err = ORA_OK;
  for (int64_t i = 0; i < n; ++i) {
    int64_t c[3] = {0, 0, 0};
    for (int k = 0; k < g->dim; ++k) {
      c[k] = cell_coord(x[3 * i + k], g->lo[k], g->cs);
      if (c[k] < 1 || c[k] > g->nc[k] - 2) err = ORA_E_NUMERIC;
      if (c[k] < 0) c[k] = 0;
      if (c[k] > g->nc[k] - 1) c[k] = g->nc[k] - 1;
    }
    int64_t id = (c[2] * g->nc[1] + c[1]) * g->nc[0] + c[0];
    g->next[i] = g->head[id];
    g->head[id] = i;
  }
  return err;
}

/* All particles of the 3^dim cells around point p; -1 if p is outside. */
static int gather(const grid_t* g, const double* p, int64_t* out) {
  int64_t c[3] = {0, 0, 0};
  for (int k = 0; k < g->dim; ++k) {
    c[k] = cell_coord(p[k], g->lo[k], g->cs);
    if (c[k] < 1 || c[k] > g->nc[k] - 2) return -1;
  }
  int m = 0;
  int zr = g->dim == 3 ? 1 : 0;
  for (int dz = -zr; dz <= zr; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        int64_t id = ((c[2] + dz) * g->nc[1] + (c[1] + dy)) * g->nc[0] + (c[0] + dx);
        for (int64_t j = g->head[id]; j >= 0; j = g->next[j]) {
          if (m >= MAXNB) return -1;
          out[m++] = j;
        }
      }
  return m;
}

static double dist2(const double* a, const double* b) {
  double d0 = a[0] - b[0], d1 = a[1] - b[1], d2 = a[2] - b[2];
  return (d0 * d0 + d1 * d1) + d2 * d2;
}

static double cutoff2(const ora_params* P) {
  double rc = 2.0 * P->h;
  return rc * rc;
}

/* Neighbour set N(i) = { j != i : |x_i - x_j|^2 < (2h)^2 } (Sec. 2.2). */
static int neighbors_of(const grid_t* g, const double* x, int64_t i, double rc2,
                        int64_t* out) {
  int64_t cand[MAXNB];
  int m = gather(g, x + 3 * i, cand);
  if (m < 0) return -1;
  int k = 0;
  for (int a = 0; a < m; ++a) {
    int64_t j = cand[a];
    if (j == i) continue;
    if (dist2(x + 3 * i, x + 3 * j) < rc2) out[k++] = j;
  }
  return k;
}

static int cmp_i64(const void* a, const void* b) {
  int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  return (x > y) - (x < y);
}

int64_t ora_neighbors_brute(const ora_params* P, int64_t n, const double* x,
                            int64_t* off, int64_t* idx, int64_t cap) {
  double rc2 = cutoff2(P);
  int64_t k = 0;
  for (int64_t i = 0; i < n; ++i) {
    off[i] = k;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      if (dist2(x + 3 * i, x + 3 * j) < rc2) {
        if (k >= cap) return -1;
        idx[k++] = j;
      }
    }
  }
  off[n] = k;
  return k;
}

int64_t ora_neighbors_cll(const ora_params* P, int64_t n, const double* x,
                          int64_t* off, int64_t* idx, int64_t cap) {
  grid_t g;
  if (grid_build(&g, P, n, x) != ORA_OK) { grid_free(&g); return -1; }
  double rc2 = cutoff2(P);
  int64_t k = 0;
  int64_t nb[MAXNB];
  for (int64_t i = 0; i < n; ++i) {
    off[i] = k;
    int m = neighbors_of(&g, x, i, rc2, nb);
    if (m < 0 || k + m > cap) { grid_free(&g); return -1; }
    qsort(nb, (size_t)m, sizeof(int64_t), cmp_i64);
    memcpy(idx + k, nb, sizeof(int64_t) * (size_t)m);
    k += m;
  }
  off[n] = k;
  grid_free(&g);
  return k;
}

/* ------------------------------------------------------------------------ */
/* Buffer geometry (Secs. 2.4.1, 3.2): local frame of a buffer box.          */
/* ------------------------------------------------------------------------ */
static void to_local(const ora_buffer* b, const double* x, double* y) {
  double d0 = x[0] - b->origin[0], d1 = x[1] - b->origin[1], d2 = x[2] - b->origin[2];
  for (int k = 0; k < 3; ++k)
    y[k] = (b->frame[3 * k] * d0 + b->frame[3 * k + 1] * d1) + b->frame[3 * k + 2] * d2;
}

/* containment check of the transformed point against the reference box */
static int contained(int dim, const ora_buffer* b, const double* y) {
  if (fabs(y[1]) > b->half_width[0]) return 0;
  if (dim == 3 && fabs(y[2]) > b->half_width[1]) return 0;
  return 1;
}

/* region between the open face and the relabeling boundary */
static int in_region(int dim, const ora_buffer* b, const double* y) {
  return y[0] >= 0.0 && y[0] <= b->length && contained(dim, b, y);
}

/* start-up ramp of a buffer's prescribed values: 0.5 (1 - cos(pi t / T)) */
static double ramp(const ora_buffer* b, double t) {
  if (b->ramp_time > 0.0 && t < b->ramp_time) return 0.5 * (1.0 - cos(PI * t / b->ramp_time));
  return 1.0;
}

static const ora_buffer* find_buffer(const ora_buffer* B, int nbuf, int id) {
  for (int q = 0; q < nbuf; ++q)
    if (B[q].id == id) return &B[q];
  return NULL;
}

static int is_real(uint32_t t) { return KIND(t) == ORA_FLUID || KIND(t) == ORA_BUFFER; }

static double pow_dim(double a, int dim) { return dim == 2 ? a * a : a * a * a; }

/* ------------------------------------------------------------------------ */
/* Correction matrix, Eq. (equ-B-matrix), with the mirror boundary treatment */
/* of Sec. 3.3: near each buffer's open face the mirror images of the real   */
/* particles (self included) across the face plane complete the support.     */
/* ------------------------------------------------------------------------ */
/* B = A^-1 with a guard for ill-conditioned moments (paper silent; reading):
 * with d = det A / (tr A / dim)^dim (1 for an isotropic support, >= 0.5 for
 * every healthy, truncated or jittered support), B = A^-1 for d >= 0.25 and
 * B = w A^-1 + (1 - w) I, w = (d / 0.25)^2, below; B = I if tr A <= 0 or
 * d <= 0 (fewer than dim independent neighbours). */
static void invert_guarded(int dim, const double* A, double* Bm) {
  const double theta = 0.25;
  double inv[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  double tr, det, d;
  for (int a = 0; a < 9; ++a) Bm[a] = 0.0;
  if (dim == 2) {
    tr = A[0] + A[4];
    det = A[0] * A[4] - A[1] * A[3];
    d = (tr > 0.0) ? det / ((0.5 * tr) * (0.5 * tr)) : 0.0;
    if (!(tr > 0.0) || !(d > 0.0)) {
      Bm[0] = Bm[4] = 1.0;
      return;
    }
    inv[0] = A[4] / det;
    inv[1] = -A[1] / det;
    inv[3] = -A[3] / det;
    inv[4] = A[0] / det;
  } else {
    double c00 = A[4] * A[8] - A[5] * A[7];
    double c01 = A[5] * A[6] - A[3] * A[8];
    double c02 = A[3] * A[7] - A[4] * A[6];
    det = A[0] * c00 + A[1] * c01 + A[2] * c02;
    tr = A[0] + A[4] + A[8];
    double t3 = tr / 3.0;
    d = (tr > 0.0) ? det / (t3 * t3 * t3) : 0.0;
    if (!(tr > 0.0) || !(d > 0.0)) {
      Bm[0] = Bm[4] = Bm[8] = 1.0;
      return;
    }
    inv[0] = c00 / det;
    inv[1] = (A[2] * A[7] - A[1] * A[8]) / det;
    inv[2] = (A[1] * A[5] - A[2] * A[4]) / det;
    inv[3] = c01 / det;
    inv[4] = (A[0] * A[8] - A[2] * A[6]) / det;
    inv[5] = (A[2] * A[3] - A[0] * A[5]) / det;
    inv[6] = c02 / det;
    inv[7] = (A[1] * A[6] - A[0] * A[7]) / det;
    inv[8] = (A[0] * A[4] - A[1] * A[3]) / det;
  }
  double w = d >= theta ? 1.0 : (d / theta) * (d / theta);
  for (int a = 0; a < 9; ++a) {
    double id = (a % 4 == 0 && (a < 8 || dim == 3)) ? 1.0 : 0.0;
    Bm[a] = w * inv[a] + (1.0 - w) * id;
  }
}

/* A_i -= V_j r_ij (x) grad W_ij */
static void add_moment(int dim, double h, double* A, const double* r, double r2,
                       double Vj) {
  double f = kernel_dW_over_r(sqrt(r2), h, dim);
  for (int a = 0; a < dim; ++a)
    for (int b = 0; b < dim; ++b) A[3 * a + b] -= Vj * r[a] * (f * r[b]);
}

/* Enumerate the mirror images seen by particle i.  Calls back per image. */
typedef void (*ghost_fn)(void* ctx, const double* img, double Vj);

static int for_ghosts(const ora_params* P, const ora_buffer* B, int nbuf,
                      const ora_state* S, const double* vol, const grid_t* g,
                      int64_t i, ghost_fn fn, void* ctx) {
  int dim = P->dim;
  double rc2 = cutoff2(P);
  double twoh = 2.0 * P->h;
  const double* xi = S->x + 3 * i;
  int64_t cand[MAXNB];
  for (int q = 0; q < nbuf; ++q) {
    const ora_buffer* b = &B[q];
    double yi[3];
    to_local(b, xi, yi);
    if (!(yi[0] >= 0.0 && yi[0] < twoh)) continue;
    double t = 2.0 * yi[0];
    double m[3];
    for (int k = 0; k < 3; ++k) m[k] = xi[k] - t * b->frame[k];
    int nc = gather(g, m, cand);
    if (nc < 0) return ORA_E_NUMERIC;
    for (int a = 0; a < nc; ++a) {
      int64_t j = cand[a];
      if (!is_real(S->tag[j])) continue;
      double yj[3];
      to_local(b, S->x + 3 * j, yj);
      if (!(yj[0] >= 0.0) || !contained(dim, b, yj)) continue;
      double tj = 2.0 * yj[0];
      double img[3];
      for (int k = 0; k < 3; ++k) img[k] = S->x[3 * j + k] - tj * b->frame[k];
      if (dist2(xi, img) < rc2) fn(ctx, img, vol[j]);
    }
  }
  return ORA_OK;
}

typedef struct {
  int dim;
  double h;
  const double* xi;
  double* A;
  double* sW;
} moment_ctx;

static void ghost_moment(void* c, const double* img, double Vj) {
  moment_ctx* m = (moment_ctx*)c;
  double r[3] = {m->xi[0] - img[0], m->xi[1] - img[1], m->xi[2] - img[2]};
  double r2 = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
  add_moment(m->dim, m->h, m->A, r, r2, Vj);
  if (m->sW) *m->sW += ora_kernel_W(sqrt(r2), m->h, m->dim) * Vj;
}

static void volumes(const ora_params* P, const ora_state* S, double* vol) {
  double Vw = pow_dim(P->dp, P->dim);
  double m = P->rho0 * Vw;
  for (int64_t i = 0; i < S->n; ++i)
    vol[i] = KIND(S->tag[i]) == ORA_WALL ? Vw : m / S->rho[i];
}

static int correction_impl(const ora_params* P, const ora_buffer* B, int nbuf,
                           const ora_state* S, const double* vol, const grid_t* g,
                           int mirror, double* Bmat, double* sumW) {
  int dim = P->dim;
  double h = P->h, rc2 = cutoff2(P);
  int err = ORA_OK;
#pragma omp parallel for schedule(dynamic, 64) num_threads(g_threads)
  for (int64_t i = 0; i < S->n; ++i) {
    double A[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    double sW = ora_kernel_W(0.0, h, dim) * vol[i];
    int64_t nb[MAXNB];
    if (!is_real(S->tag[i])) {
      for (int a = 0; a < 9; ++a) Bmat[9 * i + a] = (a % 4 == 0 && (a < 8 || dim == 3)) ? 1.0 : 0.0;
      if (sumW) sumW[i] = 0.0;
      continue;
    }
    int m = neighbors_of(g, S->x, i, rc2, nb);
    if (m < 0) { err = ORA_E_NUMERIC; continue; }
    const double* xi = S->x + 3 * i;
    for (int a = 0; a < m; ++a) {
      int64_t j = nb[a];
      double r[3] = {xi[0] - S->x[3 * j], xi[1] - S->x[3 * j + 1], xi[2] - S->x[3 * j + 2]};
      double r2 = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
      add_moment(dim, h, A, r, r2, vol[j]);
      sW += ora_kernel_W(sqrt(r2), h, dim) * vol[j];
    }
    if (mirror) {
      moment_ctx mc = {dim, h, xi, A, &sW};
      if (for_ghosts(P, B, nbuf, S, vol, g, i, ghost_moment, &mc) != ORA_OK)
        err = ORA_E_NUMERIC;
    }
    invert_guarded(dim, A, Bmat + 9 * i);
    if (sumW) sumW[i] = sW;
  }
  return err;
}

int ora_correction(const ora_params* P, const ora_buffer* B, int nbuf,
                   const ora_state* S, int mirror, double* Bmat, double* sumW) {
  grid_t g;
  int err = grid_build(&g, P, S->n, S->x);
  double* vol = (double*)malloc(sizeof(double) * (size_t)(S->n + 1));
  volumes(P, S, vol);
  if (err == ORA_OK) err = correction_impl(P, B, nbuf, S, vol, &g, mirror, Bmat, sumW);
  free(vol);
  grid_free(&g);
  return err;
}

typedef struct {
  double* gx;
  double* gv;
  int64_t n, cap;
} ghost_list;

static void ghost_collect(void* c, const double* img, double Vj) {
  ghost_list* L = (ghost_list*)c;
  if (L->n < L->cap) {
    for (int k = 0; k < 3; ++k) L->gx[3 * L->n + k] = img[k];
    L->gv[L->n] = Vj;
  }
  L->n++;
}

int64_t ora_ghosts(const ora_params* P, const ora_buffer* B, int nbuf,
                   const ora_state* S, int64_t i, double* gx, double* gvol,
                   int64_t cap) {
  grid_t g;
  if (grid_build(&g, P, S->n, S->x) != ORA_OK) { grid_free(&g); return -1; }
  double* vol = (double*)malloc(sizeof(double) * (size_t)(S->n + 1));
  volumes(P, S, vol);
  ghost_list L = {gx, gvol, 0, cap};
  int err = for_ghosts(P, B, nbuf, S, vol, &g, i, ghost_collect, &L);
  free(vol);
  grid_free(&g);
  return err == ORA_OK ? L.n : -1;
}

/* ------------------------------------------------------------------------ */
/* Pair operators of Sec. 2.2 on one state.                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
  const ora_params* P;
  const ora_buffer* B;
  int nbuf;
  const ora_state* S;
  const grid_t* g;
  const double* rho;   /* density used for the 1/rho_i and 2 rho_i factors */
  const double* p;     /* effective pressure */
  const double* vol;
  const double* Bmat;
  const double* x;
  const double* v;
  double t;            /* time of the prescribed boundary values */
} pass_t;

/* Equation of state, Eq. (eos), and Table 1: p_eff = p + 2/3 rho k (RANS). */
static double eos(const ora_params* P, double rho, double k) {
  double p = P->rho0 * P->c0 * P->c0 * (rho / P->rho0 - 1.0);
  if (P->turbulence) p += (2.0 / 3.0) * rho * k;
  return p;
}

static void matvec(const double* M, const double* a, double* out) {
  for (int r = 0; r < 3; ++r)
    out[r] = (M[3 * r] * a[0] + M[3 * r + 1] * a[1]) + M[3 * r + 2] * a[2];
}

/* Pressure acceleration: Eq. (eq-discretize-momentum-p-RKGC) for the pair
 * sum and Eq. (eq-pressure-gradient-obc-B-final) for the open-boundary
 * compensation of buffer particles (Table 2 selects the variant). */
static int pass_pressure(const pass_t* T, double* ap, int64_t* npairs) {
  const ora_params* P = T->P;
  int dim = P->dim, mode = P->obc_mode;
  int useB = mode >= 2, compB = mode == 4;
  double h = P->h, rc2 = cutoff2(P);
  int err = ORA_OK;
  int64_t pairs = 0;
#pragma omp parallel for schedule(dynamic, 64) num_threads(g_threads) reduction(+ : pairs)
  for (int64_t i = 0; i < T->S->n; ++i) {
    double acc[3] = {0, 0, 0}, s[3] = {0, 0, 0};
    int64_t nb[MAXNB];
    if (!is_real(T->S->tag[i])) { ap[3 * i] = ap[3 * i + 1] = ap[3 * i + 2] = 0.0; continue; }
    int m = neighbors_of(T->g, T->x, i, rc2, nb);
    if (m < 0) { err = ORA_E_NUMERIC; continue; }
    pairs += m;
    const double* xi = T->x + 3 * i;
    const double* Bi = T->Bmat + 9 * i;
    double pi = T->p[i];
    for (int a = 0; a < m; ++a) {
      int64_t j = nb[a];
      double r[3] = {xi[0] - T->x[3 * j], xi[1] - T->x[3 * j + 1], xi[2] - T->x[3 * j + 2]};
      double r2 = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
      double f = kernel_dW_over_r(sqrt(r2), h, dim);
      double gW[3] = {f * r[0], f * r[1], f * r[2]};
      int wall = KIND(T->S->tag[j]) == ORA_WALL;
      double Vj = T->vol[j];
      double pj = wall ? pi : T->p[j];
      const double* Bj = wall ? Bi : T->Bmat + 9 * j;
      double term[3];
      if (useB) {
        double bj[3], bi[3];
        matvec(Bj, gW, bj);
        matvec(Bi, gW, bi);
        for (int k = 0; k < 3; ++k) term[k] = pi * bj[k] + pj * bi[k];
      } else {
        for (int k = 0; k < 3; ++k) term[k] = (pi + pj) * gW[k];
      }
      for (int k = 0; k < 3; ++k) {
        acc[k] += Vj * term[k];
        s[k] += Vj * gW[k];
      }
    }
    uint32_t t = T->S->tag[i];
    if (KIND(t) == ORA_BUFFER) {
      const ora_buffer* b = find_buffer(T->B, T->nbuf, BID(t));
      if (b && b->p_mode != ORA_P_NONE) {
        double pob = b->p_mode == ORA_P_PRESCRIBED ? b->p_ob * ramp(b, T->t) : pi;
        double c[3];
        if (compB) matvec(Bi, s, c);
        else { c[0] = s[0]; c[1] = s[1]; c[2] = s[2]; }
        for (int k = 0; k < 3; ++k) acc[k] -= 2.0 * pob * c[k];
      }
    }
    for (int k = 0; k < 3; ++k) ap[3 * i + k] = -acc[k] / T->rho[i];
  }
  if (npairs) *npairs += pairs;
  return err;
}

/* Continuity with the low-dissipation Riemann solver,
 * Eqs. (discretize-continuity-equ-riemann) and (eq-intermediate-vel). */
static int pass_density(const pass_t* T, double* drho, int64_t* npairs) {
  const ora_params* P = T->P;
  int dim = P->dim;
  double h = P->h, rc2 = cutoff2(P);
  double rc0 = P->rho0 * P->c0;
  int err = ORA_OK;
  int64_t pairs = 0;
#pragma omp parallel for schedule(dynamic, 64) num_threads(g_threads) reduction(+ : pairs)
  for (int64_t i = 0; i < T->S->n; ++i) {
    int64_t nb[MAXNB];
    if (!is_real(T->S->tag[i])) { drho[i] = 0.0; continue; }
    int m = neighbors_of(T->g, T->x, i, rc2, nb);
    if (m < 0) { err = ORA_E_NUMERIC; continue; }
    pairs += m;
    const double* xi = T->x + 3 * i;
    const double* vi = T->v + 3 * i;
    double pi = T->p[i];
    double sum = 0.0;
    for (int a = 0; a < m; ++a) {
      int64_t j = nb[a];
      double r[3] = {xi[0] - T->x[3 * j], xi[1] - T->x[3 * j + 1], xi[2] - T->x[3 * j + 2]};
      double r2 = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
      double rr = sqrt(r2);
      if (!(rr > 0.0)) continue;
      double f = kernel_dW_over_r(rr, h, dim);
      double gW[3] = {f * r[0], f * r[1], f * r[2]};
      int wall = KIND(T->S->tag[j]) == ORA_WALL;
      double vj[3] = {0, 0, 0};
      if (!wall) { vj[0] = T->v[3 * j]; vj[1] = T->v[3 * j + 1]; vj[2] = T->v[3 * j + 2]; }
      double pj = wall ? pi : T->p[j];
      double e[3] = {-r[0] / rr, -r[1] / rr, -r[2] / rr};
      double vbar[3] = {0.5 * (vi[0] + vj[0]), 0.5 * (vi[1] + vj[1]), 0.5 * (vi[2] + vj[2])};
      double Ubar = (vbar[0] * e[0] + vbar[1] * e[1]) + vbar[2] * e[2];
      double Ustar = Ubar + (pi - pj) / (2.0 * rc0);
      double dv[3];
      for (int k = 0; k < 3; ++k) {
        double vstar = Ustar * e[k] + (vbar[k] - Ubar * e[k]);
        dv[k] = vi[k] - vstar;
      }
      sum += T->vol[j] * ((dv[0] * gW[0] + dv[1] * gW[1]) + dv[2] * gW[2]);
    }
    drho[i] = 2.0 * T->rho[i] * sum;
  }
  if (npairs) *npairs += pairs;
  return err;
}

static double nu_t_of(const ora_params* P, const ora_state* S, int64_t i) {
  if (!P->turbulence) return 0.0;
  double k = S->k[i], e = S->eps[i];
  return P->Cmu * k * k / e;
}

/* ARD viscous acceleration, Eqs. (eq-discretize-momentum-ARD2) and
 * (eq-discretize-momentum-ARD-viscosity); mu_i = rho0 nu_eff,i (Table 1). */
static int pass_viscous(const pass_t* T, double* anu, int64_t* npairs) {
  const ora_params* P = T->P;
  int dim = P->dim;
  double h = P->h, rc2 = cutoff2(P);
  int err = ORA_OK;
  int64_t pairs = 0;
#pragma omp parallel for schedule(dynamic, 64) num_threads(g_threads) reduction(+ : pairs)
  for (int64_t i = 0; i < T->S->n; ++i) {
    int64_t nb[MAXNB];
    double a3[3] = {0, 0, 0};
    if (!is_real(T->S->tag[i])) { anu[3 * i] = anu[3 * i + 1] = anu[3 * i + 2] = 0.0; continue; }
    int m = neighbors_of(T->g, T->x, i, rc2, nb);
    if (m < 0) { err = ORA_E_NUMERIC; continue; }
    pairs += m;
    const double* xi = T->x + 3 * i;
    const double* vi = T->v + 3 * i;
    double mu_i = P->rho0 * (P->nu_l + nu_t_of(P, T->S, i));
    for (int a = 0; a < m; ++a) {
      int64_t j = nb[a];
      double r[3] = {xi[0] - T->x[3 * j], xi[1] - T->x[3 * j + 1], xi[2] - T->x[3 * j + 2]};
      double r2 = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
      double rr = sqrt(r2);
      double f = kernel_dW_over_r(rr, h, dim);
      int wall = KIND(T->S->tag[j]) == ORA_WALL;
      double vij[3];
      for (int k = 0; k < 3; ++k) vij[k] = vi[k] - (wall ? -vi[k] : T->v[3 * j + k]);
      double mu_j = wall ? mu_i : P->rho0 * (P->nu_l + nu_t_of(P, T->S, j));
      double mu_h = 2.0 * mu_i * mu_j / (mu_i + mu_j);
      double beta = 0.0;
      if (P->turbulence && rr > 0.0) {
        double ve = -((vij[0] * r[0] + vij[1] * r[1]) + vij[2] * r[2]) / rr;
        beta = fmin(P->eta * fmax(ve, 0.0), P->c0);
      }
      double mu_R = 0.5 * P->rho0 * h * beta;
      double mu_ad = fmax(mu_h, mu_R);
      for (int k = 0; k < 3; ++k) a3[k] += mu_ad * vij[k] * f * T->vol[j];
    }
    for (int k = 0; k < 3; ++k) anu[3 * i + k] = 2.0 / T->rho[i] * a3[k];
  }
  if (npairs) *npairs += pairs;
  return err;
}

/* Transport-velocity shift (Sec. 2.3 names the transport-velocity
 * formulation for particle regularity and cites it without a formula; this
 * is the standard position-correction form, stated here):
 *   dx_i = -alpha h^2 sum_j 2 V_j grad_i W_ij
 * over every neighbour j (fluid, buffer, wall) of a particle i that moves
 * with the flow: a FLUID particle, or a BUFFER particle of a buffer whose
 * velocity is extrapolated from the fluid (Table 3); zero for particles of
 * prescribed-velocity buffers and for walls.  A buffer particle keeps only
 * the component tangential to its buffer's open face (normal n_b removed):
 * its support is cut at the face, where the sum would push it out, and its
 * motion across the face, which decides deletion and injection, is the
 * buffer's own; within 2h of the ends of the box's transverse extent (a
 * corner of the domain, where the support is cut along the face too) it
 * gets none.  The sum vanishes on a uniform lattice and
 * points from i towards denser neighbours, so dx_i moves particles towards
 * emptier space.  It is evaluated on the start-of-step configuration and
 * added to the position at the end of the advection step: over the step the
 * particle travels with v + dx / dt_adv. */
static int pass_shift(const pass_t* T, double* dx) {
  const ora_params* P = T->P;
  int dim = P->dim;
  double h = P->h, rc2 = cutoff2(P);
  double c = -P->tvf_alpha * h * h;
  int err = ORA_OK;
#pragma omp parallel for schedule(dynamic, 64) num_threads(g_threads)
  for (int64_t i = 0; i < T->S->n; ++i) {
    int64_t nb[MAXNB];
    double s3[3] = {0, 0, 0};
    dx[3 * i] = dx[3 * i + 1] = dx[3 * i + 2] = 0.0;
    uint32_t ti = T->S->tag[i];
    const ora_buffer* b = NULL;
    if (KIND(ti) == ORA_BUFFER) {
      b = find_buffer(T->B, T->nbuf, BID(ti));
      if (!b || b->vel_mode != ORA_VEL_EXTRAPOLATE) continue;
    } else if (KIND(ti) != ORA_FLUID) {
      continue;
    }
    int m = neighbors_of(T->g, T->x, i, rc2, nb);
    if (m < 0) { err = ORA_E_NUMERIC; continue; }
    const double* xi = T->x + 3 * i;
    for (int a = 0; a < m; ++a) {
      int64_t j = nb[a];
      double r[3] = {xi[0] - T->x[3 * j], xi[1] - T->x[3 * j + 1], xi[2] - T->x[3 * j + 2]};
      double r2 = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
      double f = kernel_dW_over_r(sqrt(r2), h, dim);   /* grad_i W_ij = f r_ij */
      for (int k = 0; k < dim; ++k) s3[k] += 2.0 * T->vol[j] * f * r[k];
    }
    for (int k = 0; k < dim; ++k) dx[3 * i + k] = c * s3[k];
    if (b) {   /* tangential part only: dx - (dx . n_b) n_b; none near the ends */
      double y[3];
      to_local(b, xi, y);
      int end = fabs(y[1]) > b->half_width[0] - 2.0 * h ||
                (dim == 3 && fabs(y[2]) > b->half_width[1] - 2.0 * h);
      const double* nb_ = b->frame;
      double dn = (dx[3 * i] * nb_[0] + dx[3 * i + 1] * nb_[1]) + dx[3 * i + 2] * nb_[2];
      for (int k = 0; k < dim; ++k) dx[3 * i + k] = end ? 0.0 : dx[3 * i + k] - dn * nb_[k];
    }
  }
  return err;
}

/* Velocity gradient, Eq. (velo-grad-equ), and the k-epsilon rates,
 * Eqs. (k-discretized-equ), (epsilon-discretized-equ) with
 * G_k = tau_t : grad v, tau_t = nu_t (grad v + grad v^T) - 2k I / 3. */
static int pass_turbulence(const pass_t* T, double* gradv, double* dk, double* de) {
  const ora_params* P = T->P;
  const ora_state* S = T->S;
  int dim = P->dim;
  double h = P->h, rc2 = cutoff2(P);
  int err = ORA_OK;
#pragma omp parallel for schedule(dynamic, 64) num_threads(g_threads)
  for (int64_t i = 0; i < S->n; ++i) {
    int64_t nb[MAXNB];
    double G[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (!is_real(S->tag[i])) {
      for (int a = 0; a < 9; ++a) gradv[9 * i + a] = 0.0;
      dk[i] = de[i] = 0.0;
      continue;
    }
    int m = neighbors_of(T->g, T->x, i, rc2, nb);
    if (m < 0) { err = ORA_E_NUMERIC; continue; }
    const double* xi = T->x + 3 * i;
    const double* vi = T->v + 3 * i;
    const double* Bi = T->Bmat + 9 * i;
    double ki = S->k[i], ei = S->eps[i];
    double nti = nu_t_of(P, S, i);
    double Dk_i = P->nu_l + nti / P->sigma_k, De_i = P->nu_l + nti / P->sigma_eps;
    double diff_k = 0.0, diff_e = 0.0;
    for (int a = 0; a < m; ++a) {
      int64_t j = nb[a];
      double r[3] = {xi[0] - T->x[3 * j], xi[1] - T->x[3 * j + 1], xi[2] - T->x[3 * j + 2]};
      double r2 = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
      double f = kernel_dW_over_r(sqrt(r2), h, dim);
      double gW[3] = {f * r[0], f * r[1], f * r[2]};
      int wall = KIND(S->tag[j]) == ORA_WALL;
      double Vj = T->vol[j];
      double vij[3];
      for (int k = 0; k < 3; ++k) vij[k] = vi[k] - (wall ? -vi[k] : T->v[3 * j + k]);
      double BgW[3];
      matvec(Bi, gW, BgW);
      for (int a2 = 0; a2 < 3; ++a2)
        for (int b2 = 0; b2 < 3; ++b2) G[3 * a2 + b2] -= Vj * vij[a2] * BgW[b2];
      if (wall) continue;
      double ntj = nu_t_of(P, S, j);
      double Dk_j = P->nu_l + ntj / P->sigma_k, De_j = P->nu_l + ntj / P->sigma_eps;
      double Dk_h = 2.0 * Dk_i * Dk_j / (Dk_i + Dk_j);
      double De_h = 2.0 * De_i * De_j / (De_i + De_j);
      diff_k += Dk_h * (ki - S->k[j]) * f * Vj;
      diff_e += De_h * (ei - S->eps[j]) * f * Vj;
    }
    diff_k *= 2.0 / T->rho[i];
    diff_e *= 2.0 / T->rho[i];
    double dd = 0.0;
    for (int a2 = 0; a2 < 3; ++a2)
      for (int b2 = 0; b2 < 3; ++b2) dd += (G[3 * a2 + b2] + G[3 * b2 + a2]) * G[3 * a2 + b2];
    double Gk = nti * dd - (2.0 / 3.0) * ki * (G[0] + G[4] + G[8]);
    dk[i] = Gk - ei + diff_k;
    de[i] = P->C1 * (ei / ki) * Gk - P->C2 * ei * ei / ki + diff_e;
    for (int a2 = 0; a2 < 9; ++a2) gradv[9 * i + a2] = G[a2];
  }
  return err;
}

int ora_rates_eval(const ora_params* P, const ora_buffer* B, int nbuf,
                   const ora_state* S, const double* Bmat, ora_rates* R) {
  grid_t g;
  int err = grid_build(&g, P, S->n, S->x);
  if (err != ORA_OK) { grid_free(&g); return err; }
  volumes(P, S, R->vol);
  for (int64_t i = 0; i < S->n; ++i)
    R->p[i] = is_real(S->tag[i]) ? eos(P, S->rho[i], P->turbulence ? S->k[i] : 0.0) : 0.0;
  pass_t T = {P, B, nbuf, S, &g, S->rho, R->p, R->vol, Bmat, S->x, S->v, S->t};
  if (R->ap) err |= pass_pressure(&T, R->ap, NULL);
  if (R->drho) err |= pass_density(&T, R->drho, NULL);
  if (R->anu) err |= pass_viscous(&T, R->anu, NULL);
  if (P->turbulence && R->gradv && R->dk && R->deps)
    err |= pass_turbulence(&T, R->gradv, R->dk, R->deps);
  if (R->shift) err |= pass_shift(&T, R->shift);
  grid_free(&g);
  return err;
}

/* ------------------------------------------------------------------------ */
/* Time-step sizes of the dual-criteria scheme (Sec. 2.3, reading):          */
/* dt_ad = cfl_adv min(h / max(vmax, u_ref), h^2 / (2 nu_max)),              */
/* dt_ac = cfl_ac h / (c0 + vmax), n_ac = ceil(dt_ad / dt_ac).               */
/* ------------------------------------------------------------------------ */
int ora_time_step(const ora_params* P, const ora_state* S, ora_step_info* I) {
  double v2max = 0.0, numax = P->nu_l;
  for (int64_t i = 0; i < S->n; ++i) {
    if (!is_real(S->tag[i])) continue;
    const double* v = S->v + 3 * i;
    double v2 = (v[0] * v[0] + v[1] * v[1]) + v[2] * v[2];
    if (!(v2 == v2) || !(S->rho[i] == S->rho[i])) return ORA_E_NUMERIC;
    if (v2 > v2max) v2max = v2;
    double nu = P->nu_l + nu_t_of(P, S, i);
    if (nu > numax) numax = nu;
  }
  double h = P->h;
  double vmax = sqrt(v2max);
  I->vmax = vmax;
  I->numax = numax;
  I->dt_adv = P->cfl_adv * fmin(h / fmax(vmax, P->u_ref), h * h / (2.0 * numax));
  I->dt_ac = P->cfl_ac * h / (P->c0 + vmax);
  I->n_ac = (int32_t)ceil(I->dt_adv / I->dt_ac);
  if (I->n_ac < 1) I->n_ac = 1;
  return ORA_OK;
}

/* ------------------------------------------------------------------------ */
/* Buffer boundary values (Sec. 2.4.2, Table 3).                              */
/* ------------------------------------------------------------------------ */
static double profile_u(const ora_params* P, const ora_buffer* b, const double* y,
                        uint32_t pid, int64_t step, double t) {
  double w0 = b->half_width[0];
  double s = (y[1] + w0) / (2.0 * w0);
  double u;
  switch (b->profile) {
    case ORA_PROFILE_PARABOLIC:
      u = 4.0 * b->u0 * s * (1.0 - s);
      if (P->dim == 3) {
        double w1 = b->half_width[1];
        double t = (y[2] + w1) / (2.0 * w1);
        u *= 4.0 * t * (1.0 - t);
      }
      break;
    case ORA_PROFILE_SINE:
      u = 4.0 * b->u0 * s * (1.0 - s);
      for (int m = 1; m <= b->n_coef; ++m) u += b->coef[m - 1] * sin((double)m * PI * s);
      break;
    default:
      u = b->u0;
  }
  if (b->noise_amp != 0.0) u *= 1.0 + b->noise_amp * ora_uniform(P->seed, pid, step, 0);
  return u * ramp(b, t);
}

static void apply_velocity_bc(const ora_params* P, const ora_buffer* b,
                              const double* x, double* v, uint32_t pid, int64_t step,
                              double t) {
  double y[3];
  to_local(b, x, y);
  double u = profile_u(P, b, y, pid, step, t);
  for (int k = 0; k < 3; ++k) v[k] = u * b->frame[k];
}

int ora_velocity_bc(const ora_params* P, const ora_buffer* B, int nbuf, ora_state* S) {
  for (int64_t i = 0; i < S->n; ++i) {
    uint32_t t = S->tag[i];
    if (KIND(t) != ORA_BUFFER) continue;
    const ora_buffer* b = find_buffer(B, nbuf, BID(t));
    if (b && b->vel_mode == ORA_VEL_PRESCRIBED)
      apply_velocity_bc(P, b, S->x + 3 * i, S->v + 3 * i, S->pid[i], S->step, S->t);
  }
  return ORA_OK;
}

/* Density of a buffer particle with a prescribed pressure: Eq. (eos) solved
 * for p = p_ob (laminar reading of the pressure boundary value). */
static double rho_of_p(const ora_params* P, double p) {
  return P->rho0 * (p / (P->rho0 * P->c0 * P->c0) + 1.0);
}

/* ------------------------------------------------------------------------ */
/* One advection step of the dual-criteria scheme (Sec. 2.3; reading):       */
/* B, viscous force and RANS at the start-of-step state, then n_ac acoustic  */
/* kick-drift-kick sub-steps (half density update, pressure kick with the    */
/* velocity boundary condition, drift, continuity, half density update);     */
/* with tvf_alpha != 0 the transport-velocity shift of the start-of-step     */
/* state is added to the positions at the end.                               */
/* ------------------------------------------------------------------------ */
int ora_advection_step(const ora_params* P, const ora_buffer* B, int nbuf,
                       ora_state* S, double dt_adv_fixed, int n_ac_fixed,
                       ora_step_info* I) {
  int64_t n = S->n;
  int dim = P->dim;
  size_t sz = (size_t)(n + 1);
  double* Bmat = (double*)malloc(sizeof(double) * 9 * sz);
  double* vol = (double*)malloc(sizeof(double) * sz);
  double* p = (double*)malloc(sizeof(double) * sz);
  double* ap = (double*)malloc(sizeof(double) * 3 * sz);
  double* anu = (double*)malloc(sizeof(double) * 3 * sz);
  double* gradv = (double*)malloc(sizeof(double) * 9 * sz);
  double* dk = (double*)malloc(sizeof(double) * sz);
  double* de = (double*)malloc(sizeof(double) * sz);
  double* dx = P->tvf_alpha != 0.0 ? (double*)malloc(sizeof(double) * 3 * sz) : NULL;
  int err = ORA_OK;
  int64_t pairs = 0;
  grid_t g;
  ora_step_info info;
  memset(&info, 0, sizeof(info));

  err = ora_time_step(P, S, &info);
  if (err != ORA_OK) goto done;
  if (dt_adv_fixed > 0.0) {
    info.dt_adv = dt_adv_fixed;
    info.n_ac = n_ac_fixed > 0 ? n_ac_fixed : 1;
  }
  double dt = info.dt_adv / info.n_ac;

  /* advection level: correction matrix, viscous force, RANS */
  err = grid_build(&g, P, n, S->x);
  if (err != ORA_OK) { grid_free(&g); goto done; }
  volumes(P, S, vol);
  if (P->obc_mode >= 2) {
    err = correction_impl(P, B, nbuf, S, vol, &g, P->obc_mode >= 3, Bmat, NULL);
  } else {
    for (int64_t i = 0; i < n; ++i)
      for (int a = 0; a < 9; ++a) Bmat[9 * i + a] = (a == 0 || a == 4 || (a == 8 && dim == 3)) ? 1.0 : 0.0;
  }
  {
    /* pairs of the correction pass (real particles, real neighbours) */
    double rc2 = cutoff2(P);
    int64_t nb[MAXNB];
    for (int64_t i = 0; i < n; ++i)
      if (is_real(S->tag[i])) {
        int m = neighbors_of(&g, S->x, i, rc2, nb);
        if (m > 0) pairs += m;
      }
  }
  pass_t T = {P, B, nbuf, S, &g, S->rho, p, vol, Bmat, S->x, S->v, S->t};
  err |= pass_viscous(&T, anu, &pairs);
  if (dx) err |= pass_shift(&T, dx);
  if (P->turbulence) {
    err |= pass_turbulence(&T, gradv, dk, de);
    for (int64_t i = 0; i < n; ++i) {
      if (!is_real(S->tag[i])) continue;
      double k = S->k[i] + info.dt_adv * dk[i];
      double e = S->eps[i] + info.dt_adv * de[i];
      S->k[i] = fmax(k, P->k_floor);
      S->eps[i] = fmax(e, P->eps_floor);
      uint32_t t = S->tag[i];
      if (KIND(t) == ORA_BUFFER) {
        const ora_buffer* b = find_buffer(B, nbuf, BID(t));
        if (b && b->turb_mode == ORA_TURB_FREESTREAM) {
          S->k[i] = b->k_bc;
          S->eps[i] = b->eps_bc;
        }
      }
    }
  }
  grid_free(&g);
  if (err != ORA_OK) goto done;

  for (int s = 0; s < info.n_ac; ++s) {
    for (int64_t i = 0; i < n; ++i) {
      if (!is_real(S->tag[i])) continue;
      S->rho[i] = S->rho[i] + 0.5 * dt * S->drho[i];
      p[i] = eos(P, S->rho[i], P->turbulence ? S->k[i] : 0.0);
    }
    volumes(P, S, vol);
    err = grid_build(&g, P, n, S->x);
    if (err != ORA_OK) { grid_free(&g); goto done; }
    err = pass_pressure(&T, ap, &pairs);
    grid_free(&g);
    if (err != ORA_OK) goto done;
    for (int64_t i = 0; i < n; ++i) {
      if (!is_real(S->tag[i])) continue;
      for (int k = 0; k < dim; ++k)
        S->v[3 * i + k] = S->v[3 * i + k] + dt * (ap[3 * i + k] + anu[3 * i + k] + P->g[k]);
    }
    ora_velocity_bc(P, B, nbuf, S);
    for (int64_t i = 0; i < n; ++i) {
      if (!is_real(S->tag[i])) continue;
      for (int k = 0; k < dim; ++k) S->x[3 * i + k] = S->x[3 * i + k] + dt * S->v[3 * i + k];
    }
    err = grid_build(&g, P, n, S->x);
    if (err != ORA_OK) { grid_free(&g); goto done; }
    err = pass_density(&T, S->drho, &pairs);
    grid_free(&g);
    if (err != ORA_OK) goto done;
    for (int64_t i = 0; i < n; ++i) {
      if (!is_real(S->tag[i])) continue;
      S->rho[i] = S->rho[i] + 0.5 * dt * S->drho[i];
    }
  }
  if (dx)   /* the transport-velocity shift of the start-of-step state */
    for (int64_t i = 0; i < n; ++i)
      for (int k = 0; k < dim; ++k) S->x[3 * i + k] += dx[3 * i + k];
  S->step += 1;
  S->t += info.dt_adv;

done:
  info.n_pairs = pairs;
  if (I) *I = info;
  free(Bmat); free(vol); free(p); free(ap); free(anu); free(gradv); free(dk); free(de);
  free(dx);
  return err;
}

/* ------------------------------------------------------------------------ */
/* Buffer update (Secs. 2.4.2, 2.4.3, 3.1, 3.2).                              */
/* Per buffer b, only particles in its local cell linked list (the cells of  */
/* the global grid that cover the box, with a margin of one cell) are        */
/* examined.  From one snapshot:                                             */
/*   relabel  FLUID  in 0 <= y0 <= L_b and contained          -> BUFFER(b)   */
/*   inject   BUFFER(b), contained, y0 >= L_b + fringe (generation line)     */
/*   delete   BUFFER(b), contained, y0 < 0                                   */
/*   revert   BUFFER(b) outside b's transverse box -> FLUID, then relabel    */
/* ------------------------------------------------------------------------ */
typedef struct { int64_t lo[3], hi[3]; } cellbox;

static void lcll_box(const ora_params* P, const ora_buffer* b, cellbox* cb) {
  double cs = P->cell_size, m = cs;
  double y0s[2] = {-m, b->length + b->fringe + m};
  double y1s[2] = {-b->half_width[0] - m, b->half_width[0] + m};
  double y2s[2] = {0.0, 0.0};
  if (P->dim == 3) { y2s[0] = -b->half_width[1] - m; y2s[1] = b->half_width[1] + m; }
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int a = 0; a < 2; ++a)
    for (int c = 0; c < 2; ++c)
      for (int d = 0; d < 2; ++d)
        for (int k = 0; k < 3; ++k) {
          double gk = b->origin[k] + ((y0s[a] * b->frame[k] + y1s[c] * b->frame[3 + k]) +
                                      y2s[d] * b->frame[6 + k]);
          if (gk < lo[k]) lo[k] = gk;
          if (gk > hi[k]) hi[k] = gk;
        }
  int64_t nc[3];
  grid_dims(P, nc);
  for (int k = 0; k < 3; ++k) {
    if (k >= P->dim) { cb->lo[k] = cb->hi[k] = 0; continue; }
    int64_t a = cell_coord(lo[k], P->lo[k], cs), c = cell_coord(hi[k], P->lo[k], cs);
    if (a < 0) a = 0;
    if (c > nc[k] - 1) c = nc[k] - 1;
    cb->lo[k] = a;
    cb->hi[k] = c;
  }
}

static int in_cellbox(const ora_params* P, const cellbox* cb, const double* x) {
  for (int k = 0; k < P->dim; ++k) {
    int64_t c = cell_coord(x[k], P->lo[k], P->cell_size);
    if (c < cb->lo[k] || c > cb->hi[k]) return 0;
  }
  return 1;
}

static uint32_t decide(const ora_params* P, const ora_buffer* B, int nbuf,
                       const cellbox* boxes, const double* x, uint32_t tag) {
  int dim = P->dim;
  int kind = KIND(tag);
  double y[3];
  if (kind == ORA_BUFFER) {
    int q0 = -1;
    for (int q = 0; q < nbuf; ++q)
      if (B[q].id == BID(tag)) q0 = q;
    if (q0 < 0 || !in_cellbox(P, &boxes[q0], x)) return ORA_DEC_NONE;
    const ora_buffer* b = &B[q0];
    to_local(b, x, y);
    if (contained(dim, b, y)) {
      if (y[0] < 0.0) return ORA_DEC_DELETE | ((uint32_t)b->id << 8);
      double gen = b->length + b->fringe;
      if (y[0] >= gen) return ORA_DEC_INJECT | ((uint32_t)b->id << 8);
      return ORA_DEC_NONE;
    }
    for (int q = 0; q < nbuf; ++q) {
      if (!in_cellbox(P, &boxes[q], x)) continue;
      double y2[3];
      to_local(&B[q], x, y2);
      if (in_region(dim, &B[q], y2))
        return ORA_DEC_REVERT_RELABEL | ((uint32_t)b->id << 8) | ((uint32_t)B[q].id << 16);
    }
    /* out through the side of its box into no buffer region: if it is
     * behind the open-face plane of a buffer whose face, extended along its
     * plane by the particle's own buffer length (to the generation line) and
     * the kernel support 2h, reaches it, it has left the domain through that
     * face at a corner where two open boundaries meet, and is deleted like
     * a particle crossing a face (Sec. 2.4.3).  A face plane far away (a
     * channel bent by more than 180 degrees) does not delete it (Sec. 3.2). */
    double m = (b->length + b->fringe) + 2.0 * P->h;
    for (int q = 0; q < nbuf; ++q) {
      double y2[3];
      to_local(&B[q], x, y2);
      if (!(y2[0] < 0.0)) continue;
      if (fabs(y2[1]) > B[q].half_width[0] + m) continue;
      if (dim == 3 && fabs(y2[2]) > B[q].half_width[1] + m) continue;
      return ORA_DEC_DELETE | ((uint32_t)b->id << 8);
    }
    return ORA_DEC_REVERT | ((uint32_t)b->id << 8);
  }
  if (kind != ORA_FLUID) return ORA_DEC_NONE;
  for (int q = 0; q < nbuf; ++q) {
    if (!in_cellbox(P, &boxes[q], x)) continue;
    to_local(&B[q], x, y);
    if (in_region(dim, &B[q], y)) return ORA_DEC_RELABEL | ((uint32_t)B[q].id << 8);
  }
  return ORA_DEC_NONE;
}

static int check_buffers(const ora_buffer* B, int nbuf) {
  if (nbuf < 0 || nbuf > 255) return ORA_E_ARG;
  for (int q = 0; q < nbuf; ++q) {
    if (B[q].id < 1 || B[q].id > 255) return ORA_E_ARG;
    if (q > 0 && B[q].id <= B[q - 1].id) return ORA_E_ARG;
  }
  return ORA_OK;
}

int ora_buffer_decisions(const ora_params* P, const ora_buffer* B, int nbuf,
                         const ora_state* S, uint32_t* dec) {
  if (check_buffers(B, nbuf) != ORA_OK) return ORA_E_ARG;
  cellbox boxes[256];
  for (int q = 0; q < nbuf; ++q) lcll_box(P, &B[q], &boxes[q]);
  for (int64_t i = 0; i < S->n; ++i)
    dec[i] = decide(P, B, nbuf, boxes, S->x + 3 * i, S->tag[i]);
  return ORA_OK;
}

typedef struct { uint32_t bid, pid; int64_t i; } inj_t;

static int cmp_inj(const void* a, const void* b) {
  const inj_t* x = (const inj_t*)a;
  const inj_t* y = (const inj_t*)b;
  if (x->bid != y->bid) return x->bid < y->bid ? -1 : 1;
  return (x->pid > y->pid) - (x->pid < y->pid);
}

static void copy_particle(ora_state* S, int64_t dst, int64_t src) {
  for (int k = 0; k < 3; ++k) {
    S->x[3 * dst + k] = S->x[3 * src + k];
    S->v[3 * dst + k] = S->v[3 * src + k];
  }
  S->rho[dst] = S->rho[src];
  S->drho[dst] = S->drho[src];
  S->k[dst] = S->k[src];
  S->eps[dst] = S->eps[src];
  S->tag[dst] = S->tag[src];
  S->pid[dst] = S->pid[src];
}

int ora_buffer_update(const ora_params* P, const ora_buffer* B, int nbuf,
                      ora_state* S, ora_counts* C, const uint32_t* forced_dec) {
  if (check_buffers(B, nbuf) != ORA_OK) return ORA_E_ARG;
  int64_t n = S->n;
  uint32_t* dec = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(n + 1));
  if (forced_dec) memcpy(dec, forced_dec, sizeof(uint32_t) * (size_t)n);
  else ora_buffer_decisions(P, B, nbuf, S, dec);
  int64_t n_inj = 0;
  for (int64_t i = 0; i < n; ++i)
    if ((dec[i] & 0xFF) == ORA_DEC_INJECT) n_inj++;
  if (n + n_inj > S->cap) { free(dec); return ORA_E_CAPACITY; }
  ora_counts cnt;
  memset(&cnt, 0, sizeof(cnt));
  inj_t* inj = (inj_t*)malloc(sizeof(inj_t) * (size_t)(n_inj + 1));
  unsigned char* del = (unsigned char*)calloc((size_t)(n + n_inj + 1), 1);
  int64_t q = 0;
  for (int64_t i = 0; i < n; ++i) {
    uint32_t a = dec[i] & 0xFF, b = (dec[i] >> 8) & 0xFF, b2 = (dec[i] >> 16) & 0xFF;
    switch (a) {
      case ORA_DEC_RELABEL:
        S->tag[i] = ORA_BUFFER | (b << 8);
        cnt.n_relabel[b]++;
        break;
      case ORA_DEC_REVERT:
        S->tag[i] = ORA_FLUID;
        cnt.n_revert[b]++;
        break;
      case ORA_DEC_REVERT_RELABEL:
        S->tag[i] = ORA_BUFFER | (b2 << 8);
        cnt.n_revert[b]++;
        cnt.n_relabel[b2]++;
        break;
      case ORA_DEC_INJECT:
        inj[q].bid = b;
        inj[q].pid = S->pid[i];
        inj[q].i = i;
        q++;
        cnt.n_inject[b]++;
        break;
      case ORA_DEC_DELETE:
        del[i] = 1;
        cnt.n_delete[b]++;
        break;
      default:
        break;
    }
  }
  /* inflow: append the new fluid particles at the end of the array in the
   * canonical order (buffer id, parent pid), then recycle the parents by
   * Eq. (eq-pos-new-added) and give them the buffer's boundary values */
  qsort(inj, (size_t)n_inj, sizeof(inj_t), cmp_inj);
  for (int64_t r = 0; r < n_inj; ++r) {
    int64_t c = n + r;
    copy_particle(S, c, inj[r].i);
    S->tag[c] = ORA_FLUID;
    S->pid[c] = (uint32_t)(S->next_pid + (uint64_t)r);
  }
  for (int64_t r = 0; r < n_inj; ++r) {
    int64_t i = inj[r].i;
    const ora_buffer* b = find_buffer(B, nbuf, (int)inj[r].bid);
    for (int k = 0; k < 3; ++k) {
      double t = b->length * b->frame[k];
      S->x[3 * i + k] = S->x[3 * i + k] - t;
    }
    if (b->vel_mode == ORA_VEL_PRESCRIBED)
      apply_velocity_bc(P, b, S->x + 3 * i, S->v + 3 * i, S->pid[i], S->step, S->t);
    if (b->p_mode == ORA_P_PRESCRIBED) S->rho[i] = rho_of_p(P, b->p_ob * ramp(b, S->t));
    if (P->turbulence && b->turb_mode == ORA_TURB_FREESTREAM) {
      S->k[i] = b->k_bc;
      S->eps[i] = b->eps_bc;
    }
  }
  S->n = n + n_inj;
  S->next_pid += (uint64_t)n_inj;
  /* outflow: the overwrite-with-last while loop of Sec. 2.4.3 */
  int64_t i = 0, m = S->n;
  while (i < m) {
    if (del[i]) {
      copy_particle(S, i, m - 1);
      del[i] = del[m - 1];
      m--;
    } else {
      i++;
    }
  }
  S->n = m;
  cnt.n_real = 0;
  for (int64_t j = 0; j < S->n; ++j)
    if (is_real(S->tag[j])) cnt.n_real++;
  if (C) *C = cnt;
  free(dec);
  free(inj);
  free(del);
  return ORA_OK;
}

/* ------------------------------------------------------------------------ */
/* Objectives of the inlet-profile sensitivity study (see the header):       */
/* slab mass flux J_Q and mean wall shear stress J_tau, the latter being the  */
/* wall pairs of the viscous sum of Eq. (eq-discretize-momentum-ARD2) with    */
/* the antisymmetric dummy-wall velocity, summed over the fluid and turned    */
/* into the force on the wall.  Slab membership is an FP64 predicate taken in */
/* a fixed order without contraction.                                         */
/* ------------------------------------------------------------------------ */
int ora_objective_eval(const ora_params* P, const ora_state* S, const ora_objective* O,
                       const uint8_t* member_in, uint8_t* member_out, double J[2]) {
  if (P->turbulence || !(O->slab_width > 0.0) || !(O->wall_length > 0.0)) return ORA_E_ARG;
  int dim = P->dim;
  double Vw = pow_dim(P->dp, dim);
  double m = P->rho0 * Vw;
  double mu = P->rho0 * P->nu_l;
  double h = P->h, rc2 = cutoff2(P);
  double jq = 0.0, jt = 0.0;
  int64_t nb[MAXNB];
  grid_t g;
  int err = grid_build(&g, P, S->n, S->x);
  if (err != ORA_OK) { grid_free(&g); return err; }
  for (int64_t i = 0; i < S->n; ++i) {
    if (member_out) member_out[i] = 0;
    if (!is_real(S->tag[i])) continue;
    const double* xi = S->x + 3 * i;
    const double* vi = S->v + 3 * i;
    double s = (O->slab_normal[0] * (xi[0] - O->slab_origin[0]) +
                O->slab_normal[1] * (xi[1] - O->slab_origin[1])) +
               O->slab_normal[2] * (xi[2] - O->slab_origin[2]);
    int in = member_in ? member_in[i] != 0 : (s >= 0.0 && s < O->slab_width);
    if (member_out) member_out[i] = (uint8_t)in;
    if (in) {
      double un = (O->slab_normal[0] * vi[0] + O->slab_normal[1] * vi[1]) +
                  O->slab_normal[2] * vi[2];
      jq += m * un / O->slab_width;
    }
    double ve = (O->shear_dir[0] * vi[0] + O->shear_dir[1] * vi[1]) + O->shear_dir[2] * vi[2];
    int k = neighbors_of(&g, S->x, i, rc2, nb);
    if (k < 0) { err = ORA_E_NUMERIC; break; }
    for (int a = 0; a < k; ++a) {
      int64_t j = nb[a];
      if (KIND(S->tag[j]) != ORA_WALL) continue;
      double f = kernel_dW_over_r(sqrt(dist2(xi, S->x + 3 * j)), h, dim);
      jt -= m * (2.0 / S->rho[i]) * mu * f * Vw * (2.0 * ve);
    }
  }
  grid_free(&g);
  J[0] = jq;
  J[1] = jt / O->wall_length;
  return err;
}
