/*
 * FP64 reference implementation ("oracle") of the per-step particle pipeline
 * of the weakly compressible SPH / k-epsilon RANS method with improved
 * bidirectional open-boundary buffers (F. Wang, X. Hu, arXiv 2510.25702).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is used by the test-suite, by the
 * smoke check and by the CPU-baseline leg of the benchmark.  The product path
 * (the HIP library under paper_2510_25702_amd/) never loads, links or calls
 * it, and the two share no code, header or constant.
 *
 * Plain, slow, obviously correct: every particle sums its own neighbours in
 * FP64, neighbours are found with a cell linked list rebuilt from the current
 * positions for every pass, and every formula follows the paper's notation.
 * Each function cites the section / equation it restates.
 *
 * Parity pins: every exported operation is pinned by tests under tests/
 * (closed forms, lattice invariants, brute force); see the test files.
 */
#ifndef SPH_ORACLE_H
#define SPH_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* particle tag = kind | (buffer id << 8) */
enum { ORA_FLUID = 0, ORA_BUFFER = 1, ORA_WALL = 2, ORA_DEAD = 3 };
enum { ORA_VEL_EXTRAPOLATE = 0, ORA_VEL_PRESCRIBED = 1 };
enum { ORA_P_NONE = 0, ORA_P_PRESCRIBED = 1, ORA_P_EXTRAPOLATE = 2 };
enum { ORA_TURB_ZERO_GRADIENT = 0, ORA_TURB_FREESTREAM = 1 };
enum { ORA_PROFILE_UNIFORM = 0, ORA_PROFILE_PARABOLIC = 1, ORA_PROFILE_SINE = 2 };
/* buffer-update decision codes: action | (buffer << 8) | (new buffer << 16) */
enum { ORA_DEC_NONE = 0, ORA_DEC_RELABEL = 1, ORA_DEC_INJECT = 2,
       ORA_DEC_DELETE = 3, ORA_DEC_REVERT = 4, ORA_DEC_REVERT_RELABEL = 5 };

typedef struct {
  int32_t dim, turbulence, obc_mode, pad0;
  double dp, h, rho0, c0, nu_l, eta;
  double g[3];
  double C1, C2, Cmu, sigma_k, sigma_eps, k_floor, eps_floor;
  double cfl_adv, cfl_ac, u_ref;
  double cell_size;
  double lo[3], hi[3];
  uint64_t seed;
  double tvf_alpha;       /* transport-velocity shift coefficient; 0 = off */
} ora_params;

typedef struct {
  int32_t id, vel_mode, p_mode, turb_mode, profile, n_coef;
  double origin[3];
  double frame[9];        /* row-major; row 0 = inward unit normal n_b */
  double length;          /* L_b */
  double half_width[2];
  double fringe;          /* offset of the particle-generation line */
  double p_ob, k_bc, eps_bc, u0, noise_amp;
  double coef[16];
  double ramp_time;       /* inflow ramp 0.5 (1 - cos(pi t / ramp_time)); 0 = off */
} ora_buffer;

typedef struct {
  int64_t n, cap;
  double *x, *v;          /* [cap][3] */
  double *rho, *drho;     /* [cap]; drho = last continuity rate */
  double *k, *eps;        /* [cap] */
  uint32_t *tag, *pid;    /* [cap] */
  uint64_t next_pid;
  int64_t step;
  double t;
} ora_state;

typedef struct {
  double *p, *vol;        /* [n] effective pressure, volume m/rho */
  double *ap;             /* [n][3] pressure acceleration */
  double *drho;           /* [n] continuity rate */
  double *anu;            /* [n][3] viscous acceleration */
  double *gradv;          /* [n][9] velocity gradient (turbulent only) */
  double *dk, *deps;      /* [n] k / epsilon rates (turbulent only) */
  double *shift;          /* [n][3] transport-velocity shift (NULL: skipped) */
} ora_rates;

typedef struct {
  double dt_adv, dt_ac, vmax, numax;
  int32_t n_ac, pad;
  int64_t n_pairs;        /* directed pairs over every neighbour pass */
} ora_step_info;

typedef struct {
  int32_t n_relabel[256], n_inject[256], n_delete[256], n_revert[256];
  int64_t n_real;
} ora_counts;

/* Objectives of the inlet-profile sensitivity study (laminar runs):
 *   J_Q   = sum over real i with 0 <= n.(x_i - o) < w of m (v_i . n) / w,
 *           the mass flux through a slab of width w (per unit depth in 2D);
 *   J_tau = -(1 / L_w) sum over real i, wall j, |x_i - x_j| < 2h of
 *           m (2 / rho_i) mu f(r_ij) V_j (2 v_i . e),  f = W'(r) / r,
 *           the e-component of the viscous force that the fluid exerts on the
 *           dummy walls (antisymmetric wall velocity) per unit wall length,
 *           i.e. the mean wall shear stress; mu = rho0 nu_l. */
typedef struct {
  double slab_origin[3];  /* a point on the slab's upstream plane */
  double slab_normal[3];  /* unit normal n (flux direction) */
  double slab_width;      /* w > 0 */
  double shear_dir[3];    /* unit direction e of the wall force */
  double wall_length;     /* L_w > 0: wetted wall length (2D) or area (3D) */
} ora_objective;

/* status codes */
enum { ORA_OK = 0, ORA_E_ARG = 1, ORA_E_CAPACITY = 2, ORA_E_NUMERIC = 4 };

void     ora_set_threads(int n);
int      ora_get_threads(void);
uint64_t ora_splitmix64(uint64_t z);
double   ora_uniform(uint64_t seed, uint32_t pid, int64_t step, uint32_t comp);

double ora_kernel_W(double r, double h, int dim);
double ora_kernel_dW(double r, double h, int dim);

int64_t ora_neighbors_brute(const ora_params* P, int64_t n, const double* x,
                            int64_t* off, int64_t* idx, int64_t cap);
int64_t ora_neighbors_cll(const ora_params* P, int64_t n, const double* x,
                          int64_t* off, int64_t* idx, int64_t cap);

int ora_correction(const ora_params* P, const ora_buffer* B, int nbuf,
                   const ora_state* S, int mirror, double* Bmat, double* sumW);
int64_t ora_ghosts(const ora_params* P, const ora_buffer* B, int nbuf,
                   const ora_state* S, int64_t i, double* gx, double* gvol,
                   int64_t cap);
int ora_rates_eval(const ora_params* P, const ora_buffer* B, int nbuf,
                   const ora_state* S, const double* Bmat, ora_rates* R);
int ora_time_step(const ora_params* P, const ora_state* S, ora_step_info* I);
int ora_advection_step(const ora_params* P, const ora_buffer* B, int nbuf,
                       ora_state* S, double dt_adv_fixed, int n_ac_fixed,
                       ora_step_info* I);
int ora_buffer_decisions(const ora_params* P, const ora_buffer* B, int nbuf,
                         const ora_state* S, uint32_t* dec);
int ora_buffer_update(const ora_params* P, const ora_buffer* B, int nbuf,
                      ora_state* S, ora_counts* C, const uint32_t* forced_dec);
int ora_velocity_bc(const ora_params* P, const ora_buffer* B, int nbuf,
                    ora_state* S);
/* J[0] = J_Q, J[1] = J_tau of the current state (laminar runs only).
 * Slab membership: taken from member_in[i] (0/1) when given (a frozen event
 * of a replayed run), else from the positions; written to member_out when
 * given. */
int ora_objective_eval(const ora_params* P, const ora_state* S, const ora_objective* O,
                       const uint8_t* member_in, uint8_t* member_out, double J[2]);

#ifdef __cplusplus
}
#endif
#endif
