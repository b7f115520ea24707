/*
 * Driver that runs every exported function of the FP64 oracle on small
 * buffered cases, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_oracle_sanitizers.py).  It checks
 * nothing about the values: the sanitizers check the memory accesses and the
 * arithmetic of the oracle itself.  Exit status 0 when every call returned
 * ORA_OK.
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/sph_oracle.h"

#define CHECK(call)                                                   \
  do {                                                                \
    int st_ = (int)(call);                                            \
    if (st_ != ORA_OK) {                                              \
      fprintf(stderr, "%s:%d: %s -> %d\n", __FILE__, __LINE__, #call, st_); \
      return 1;                                                       \
    }                                                                 \
  } while (0)

static ora_params base(int dim, double dp, int turb) {
  ora_params P;
  memset(&P, 0, sizeof P);
  P.dim = dim;
  P.turbulence = turb;
  P.obc_mode = 4;
  P.dp = dp;
  P.h = 1.3 * dp;
  P.rho0 = 1.0;
  P.c0 = 10.0;
  P.nu_l = 1e-2;
  P.eta = 3.0;
  P.C1 = 1.44; P.C2 = 1.92; P.Cmu = 0.09; P.sigma_k = 1.0; P.sigma_eps = 1.3;
  P.k_floor = 1e-10; P.eps_floor = 1e-10;
  P.cfl_adv = 0.25; P.cfl_ac = 0.6; P.u_ref = 1.0;
  P.cell_size = 2.6 * P.h;
  P.seed = 7;
  P.tvf_alpha = 0.1;
  return P;
}

static ora_buffer buffer(int id, double ox, double nx, double len, double hw, int vel, int pm) {
  ora_buffer b;
  memset(&b, 0, sizeof b);
  b.id = id;
  b.vel_mode = vel;
  b.p_mode = pm;
  b.turb_mode = ORA_TURB_FREESTREAM;
  b.profile = ORA_PROFILE_SINE;
  b.n_coef = 3;
  b.coef[0] = 0.05; b.coef[1] = -0.02; b.coef[2] = 0.01;
  b.u0 = 1.0;
  b.noise_amp = 0.02;
  b.origin[0] = ox; b.origin[1] = 0.5 * hw * 2.0; b.origin[2] = 0.0;
  b.frame[0] = nx; b.frame[4] = nx; b.frame[8] = 1.0;   /* rows n, t1, t2 */
  b.length = len;
  b.half_width[0] = hw; b.half_width[1] = hw;
  b.fringe = 0.05;
  b.k_bc = 1e-3; b.eps_bc = 1e-3;
  b.ramp_time = 0.5;
  return b;
}

typedef struct {
  ora_state S;
  double *x, *v, *rho, *drho, *k, *eps;
  uint32_t *tag, *pid;
} owned;

static void alloc_state(owned* o, int64_t cap) {
  o->x = calloc((size_t)cap * 3, sizeof(double));
  o->v = calloc((size_t)cap * 3, sizeof(double));
  o->rho = calloc((size_t)cap, sizeof(double));
  o->drho = calloc((size_t)cap, sizeof(double));
  o->k = calloc((size_t)cap, sizeof(double));
  o->eps = calloc((size_t)cap, sizeof(double));
  o->tag = calloc((size_t)cap, sizeof(uint32_t));
  o->pid = calloc((size_t)cap, sizeof(uint32_t));
  memset(&o->S, 0, sizeof o->S);
  o->S.cap = cap;
  o->S.x = o->x; o->S.v = o->v; o->S.rho = o->rho; o->S.drho = o->drho;
  o->S.k = o->k; o->S.eps = o->eps; o->S.tag = o->tag; o->S.pid = o->pid;
}

static void free_state(owned* o) {
  free(o->x); free(o->v); free(o->rho); free(o->drho);
  free(o->k); free(o->eps); free(o->tag); free(o->pid);
}

static void add(owned* o, double x, double y, double z, uint32_t tag) {
  int64_t i = o->S.n++;
  o->x[3 * i] = x; o->x[3 * i + 1] = y; o->x[3 * i + 2] = z;
  o->rho[i] = 1.0;
  o->tag[i] = tag;
  o->pid[i] = (uint32_t)i;
  if (tag == ORA_FLUID) { o->k[i] = 1e-3; o->eps[i] = 1e-3; o->v[3 * i] = 0.1; }
  o->S.next_pid = (uint64_t)i + 1;
}

/* 2D channel [0, L] x [0, H] with walls above and below, a velocity inlet
 * and a pressure outlet; laminar or k-epsilon. */
static int run_channel(int turb) {
  const double dp = 0.1, L = 4.0, H = 1.0;
  ora_params P = base(2, dp, turb);
  ora_buffer B[2] = {buffer(1, 0.0, 1.0, 4 * dp, 0.5 * H, ORA_VEL_PRESCRIBED, ORA_P_NONE),
                     buffer(2, L, -1.0, 4 * dp, 0.5 * H, ORA_VEL_EXTRAPOLATE, ORA_P_PRESCRIBED)};
  owned o;
  alloc_state(&o, 2000);
  for (int i = 0; i < 40; ++i)
    for (int j = 0; j < 10; ++j) add(&o, (i + 0.5) * dp, (j + 0.5) * dp, 0.0, ORA_FLUID);
  for (int i = -4; i < 44; ++i)
    for (int l = 0; l < 3; ++l) {
      add(&o, (i + 0.5) * dp, -(l + 0.5) * dp, 0.0, ORA_WALL);
      add(&o, (i + 0.5) * dp, H + (l + 0.5) * dp, 0.0, ORA_WALL);
    }
  P.lo[0] = -1.5; P.lo[1] = -1.5; P.lo[2] = -P.cell_size;
  P.hi[0] = L + 1.5; P.hi[1] = H + 1.5; P.hi[2] = P.cell_size;
  ora_counts cnt;
  CHECK(ora_buffer_update(&P, B, 2, &o.S, &cnt, NULL));
  int64_t n = o.S.n;
  double* Bm = calloc((size_t)n * 9, sizeof(double));
  double* sW = calloc((size_t)n, sizeof(double));
  CHECK(ora_correction(&P, B, 2, &o.S, 1, Bm, sW));
  ora_rates R;
  R.p = calloc((size_t)n, sizeof(double));
  R.vol = calloc((size_t)n, sizeof(double));
  R.ap = calloc((size_t)n * 3, sizeof(double));
  R.drho = calloc((size_t)n, sizeof(double));
  R.anu = calloc((size_t)n * 3, sizeof(double));
  R.gradv = calloc((size_t)n * 9, sizeof(double));
  R.dk = calloc((size_t)n, sizeof(double));
  R.deps = calloc((size_t)n, sizeof(double));
  R.shift = calloc((size_t)n * 3, sizeof(double));
  CHECK(ora_rates_eval(&P, B, 2, &o.S, Bm, &R));
  double gx[3 * 256], gv[256];
  if (ora_ghosts(&P, B, 2, &o.S, 5, gx, gv, 256) < 0) return 1;
  int64_t* off = calloc((size_t)n + 1, sizeof(int64_t));
  int64_t* idx = calloc((size_t)n * 64, sizeof(int64_t));
  if (ora_neighbors_brute(&P, n, o.x, off, idx, n * 64) < 0) return 1;
  if (ora_neighbors_cll(&P, n, o.x, off, idx, n * 64) < 0) return 1;
  ora_step_info I;
  CHECK(ora_time_step(&P, &o.S, &I));
  for (int s = 0; s < 4; ++s) {
    /* push the inlet buffer forward so that injections happen */
    for (int64_t i = 0; i < o.S.n; ++i)
      if ((o.tag[i] & 3u) == ORA_BUFFER && ((o.tag[i] >> 8) & 0xFFu) == 1) o.x[3 * i] += 0.3 * dp;
    CHECK(ora_advection_step(&P, B, 2, &o.S, 0.0, 0, &I));
    uint32_t* dec = calloc((size_t)o.S.n, sizeof(uint32_t));
    CHECK(ora_buffer_decisions(&P, B, 2, &o.S, dec));
    free(dec);
    CHECK(ora_buffer_update(&P, B, 2, &o.S, &cnt, NULL));
  }
  CHECK(ora_velocity_bc(&P, B, 2, &o.S));
  if (!turb) {
    ora_objective O;
    memset(&O, 0, sizeof O);
    O.slab_origin[0] = L - 8 * dp; O.slab_normal[0] = 1.0; O.slab_width = 4 * dp;
    O.shear_dir[0] = 1.0; O.wall_length = 2.0 * L;
    uint8_t* mem = calloc((size_t)o.S.n, 1);
    double J[2];
    CHECK(ora_objective_eval(&P, &o.S, &O, NULL, mem, J));
    CHECK(ora_objective_eval(&P, &o.S, &O, mem, NULL, J));
    free(mem);
  }
  free(off); free(idx); free(Bm); free(sW);
  free(R.p); free(R.vol); free(R.ap); free(R.drho); free(R.anu); free(R.gradv);
  free(R.dk); free(R.deps); free(R.shift);
  free_state(&o);
  return 0;
}

/* 3D duct block with an inlet and an outlet buffer, one step. */
static int run_duct(void) {
  const double dp = 0.1;
  ora_params P = base(3, dp, 0);
  ora_buffer B[2] = {buffer(1, 0.0, 1.0, 4 * dp, 0.4, ORA_VEL_PRESCRIBED, ORA_P_NONE),
                     buffer(2, 2.0, -1.0, 4 * dp, 0.4, ORA_VEL_EXTRAPOLATE, ORA_P_PRESCRIBED)};
  for (int q = 0; q < 2; ++q) { B[q].origin[1] = 0.4; B[q].origin[2] = 0.4; B[q].profile = ORA_PROFILE_PARABOLIC; }
  owned o;
  alloc_state(&o, 6000);
  for (int i = 0; i < 20; ++i)
    for (int j = 0; j < 8; ++j)
      for (int k = 0; k < 8; ++k)
        add(&o, (i + 0.5) * dp, (j + 0.5) * dp, (k + 0.5) * dp, ORA_FLUID);
  for (int d = 0; d < 3; ++d) { P.lo[d] = -1.0; P.hi[d] = 3.0; }
  ora_counts cnt;
  CHECK(ora_buffer_update(&P, B, 2, &o.S, &cnt, NULL));
  ora_step_info I;
  CHECK(ora_advection_step(&P, B, 2, &o.S, 0.0, 0, &I));
  CHECK(ora_buffer_update(&P, B, 2, &o.S, &cnt, NULL));
  free_state(&o);
  return 0;
}

int main(void) {
  ora_set_threads(1);
  if (run_channel(0)) return 1;
  if (run_channel(1)) return 1;
  if (run_duct()) return 1;
  printf("oracle sanitizer run ok\n");
  return 0;
}
