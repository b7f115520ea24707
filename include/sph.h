/*
 * sph.h - C ABI of the MI355X (gfx950) implementation of the per-step
 * particle pipeline of the weakly compressible SPH / k-epsilon RANS method
 * with improved bidirectional open-boundary buffers
 * (F. Wang, X. Hu, "An efficient implementation of the bidirectional buffer:
 *  towards laminar and turbulent open-boundary flows", arXiv 2510.25702).
 *
 * Every function is extern "C", never throws and returns an sph_status.
 * Pointers marked "device" are HIP device pointers on the context's device;
 * all other pointers are host pointers.  The library allocates no device
 * memory: every device array it uses lives in the caller-owned workspace
 * handed to sph_create (sized by sph_workspace_size).  The only library-
 * owned memory is the host context and a small pinned host staging buffer.
 *
 * All work is enqueued on the stream given to sph_create.  Calls return
 * after enqueueing, except where a function states that it synchronises
 * with the stream (sph_step and sph_buffer_update read back a few scalars;
 * the setters and getters copy on the stream and synchronise).
 *
 * Errors: SPH_E_ARG and SPH_E_STATE are detected before any work is
 * enqueued and leave the state unchanged.  SPH_E_CAPACITY from
 * sph_buffer_update leaves the particle state unchanged.  SPH_E_NUMERIC
 * (non-finite value, particle outside the cell grid, particle displaced
 * beyond the cell skin) reports the state reached by the failing call.
 * SPH_E_HIP leaves the state undefined.  sph_last_error returns a message
 * describing the last failure of a context.
 */
#ifndef SPH_H
#define SPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SPH_OK = 0,
  SPH_E_ARG = 1,       /* invalid argument, nothing done */
  SPH_E_CAPACITY = 2,  /* particle capacity or injection limit exceeded */
  SPH_E_HIP = 3,       /* HIP runtime error */
  SPH_E_NUMERIC = 4,   /* non-finite value / particle outside grid or skin */
  SPH_E_STATE = 5      /* call out of sequence (see each function) */
} sph_status;

/* Particle tag = kind | (buffer id << 8) (Secs. 2.4.1 and 3.2: buffer
 * particles carry the identifier of their buffer). */
enum { SPH_FLUID = 0, SPH_BUFFER = 1, SPH_WALL = 2, SPH_DEAD = 3 };
enum { SPH_FP64 = 0, SPH_FP32_MIXED = 1 };
/* Buffer boundary conditions (Table 3 of the paper). */
enum { SPH_VEL_EXTRAPOLATE = 0, SPH_VEL_PRESCRIBED = 1 };
enum { SPH_P_NONE = 0, SPH_P_PRESCRIBED = 1, SPH_P_EXTRAPOLATE = 2 };
enum { SPH_TURB_ZERO_GRADIENT = 0, SPH_TURB_FREESTREAM = 1 };
enum { SPH_PROFILE_UNIFORM = 0, SPH_PROFILE_PARABOLIC = 1, SPH_PROFILE_SINE = 2 };
/* Buffer-update decision codes: action | (buffer id << 8) | (new id << 16) */
enum { SPH_DEC_NONE = 0, SPH_DEC_RELABEL = 1, SPH_DEC_INJECT = 2,
       SPH_DEC_DELETE = 3, SPH_DEC_REVERT = 4, SPH_DEC_REVERT_RELABEL = 5 };

#define SPH_MAX_BUFFERS 32
#define SPH_MAX_INJECT 4096   /* injections per sph_buffer_update */

/* Problem statement (Sec. 2: governing equations, Eq. (eos), Table 1,
 * Table A; Sec. 2.2: h = 1.3 dp).  Copied at sph_create. */
typedef struct {
  int32_t dim;          /* 2 or 3 */
  int32_t precision;    /* SPH_FP64 or SPH_FP32_MIXED (pair arithmetic) */
  int32_t turbulence;   /* 0 laminar, 1 k-epsilon RANS (Table 1) */
  int32_t obc_mode;     /* 1..4: open-boundary variant, Table 2 (4 = improved) */
  double dp;            /* particle spacing; particle mass = rho0 dp^dim */
  double h;             /* smoothing length (1.3 dp); kernel cut-off 2h */
  double rho0, c0;      /* reference density and sound speed, Eq. (eos) */
  double nu_l;          /* molecular kinematic viscosity */
  double eta;           /* ARD limiter constant (3) */
  double g[3];          /* body force */
  double C1, C2, Cmu, sigma_k, sigma_eps;   /* Table A */
  double k_floor, eps_floor;                /* lower bounds of k, epsilon */
  double cfl_adv, cfl_ac, u_ref;            /* time-step criteria */
  double cell_size;     /* cell edge, >= 2h; the margin above 2h is the skin
                           that particles may travel within one advection step */
  double lo[3], hi[3];  /* cell-grid bounds; particles must stay at least one
                           cell inside them */
  int64_t capacity;     /* particle slots: real + wall + reserve for injection */
  uint64_t seed;        /* counter-based random numbers (inlet noise) */
} sph_params;

/* One buffer (Secs. 2.4.1-2.4.3, 3.1, 3.2, Table 3).  The box is given in
 * the buffer's local frame: origin = centre of the open (outer) face; frame
 * rows are orthonormal, row 0 = unit normal n_b pointing into the fluid;
 * 0 <= y0 <= length is the relabel region, |y1| <= half_width[0] and
 * (3D) |y2| <= half_width[1] the containment box, y0 >= length + fringe the
 * particle-generation line, y0 < 0 the deletion half-space. */
typedef struct {
  int32_t id;           /* unique buffer ID, 1..255, ascending in the array */
  int32_t vel_mode;     /* SPH_VEL_* */
  int32_t p_mode;       /* SPH_P_* */
  int32_t turb_mode;    /* SPH_TURB_* */
  int32_t profile;      /* SPH_PROFILE_* (prescribed velocity along n_b) */
  int32_t n_coef;       /* sine-series coefficients used, <= 16 */
  double origin[3];
  double frame[9];      /* row-major 3x3 */
  double length;        /* L_b */
  double half_width[2];
  double fringe;        /* generation-line offset (0.5 dp in the paper) */
  double p_ob;          /* prescribed open-boundary pressure */
  double k_bc, eps_bc;  /* free-stream turbulence values */
  double u0;            /* velocity scale of the profile */
  double noise_amp;     /* relative uniform noise on the prescribed speed */
  double coef[16];      /* sine-series coefficients a_m of the profile */
  double ramp_time;     /* speed ramp 0.5 (1 - cos(pi t / ramp_time)), 0 = off */
} sph_buffer_desc;

/* Particle arrays exchanged with the caller: device pointers, FP64 / uint32,
 * component-major ([3][n] for vectors, n = count). */
typedef struct {
  double* x;     /* [3][n] position */
  double* v;     /* [3][n] velocity */
  double* rho;   /* [n] density */
  double* drho;  /* [n] last continuity rate */
  double* k;     /* [n] turbulent kinetic energy (RANS) */
  double* eps;   /* [n] dissipation rate (RANS) */
  uint32_t* tag; /* [n] kind | buffer id << 8 */
  uint32_t* pid; /* [n] persistent particle id */
} sph_particles;

/* Pair-operator outputs at the current state (device, FP64, current order). */
typedef struct {
  double* ap;     /* [3][n] pressure acceleration, Eq. (...-p-RKGC) + VIPO */
  double* drho;   /* [n] continuity rate, Eq. (...-continuity-equ-riemann) */
  double* anu;    /* [3][n] viscous acceleration, Eq. (...-ARD2) */
  double* gradv;  /* [9][n] velocity gradient (RANS only), Eq. (velo-grad-equ) */
  double* dk;     /* [n] dk/dt (RANS only), Eq. (k-discretized-equ) */
  double* deps;   /* [n] deps/dt (RANS only), Eq. (epsilon-discretized-equ) */
  double* B;      /* [9][n] correction matrix, Eq. (equ-B-matrix) */
  double* p;      /* [n] effective pressure (Table 1) */
} sph_rates;

typedef struct {
  int32_t n_relabel[256], n_inject[256], n_delete[256], n_revert[256];
  int64_t n_real;       /* fluid + buffer particles after the update */
  int64_t n_total;      /* all particles (including walls) after the update */
} sph_buffer_counts;

/* Optional override of the dual-criteria time step (frozen steps). */
typedef struct {
  double dt_adv;        /* > 0: advection step; otherwise adaptive */
  int32_t n_ac;         /* acoustic sub-steps when dt_adv > 0 */
  int32_t pad;
} sph_step_ctrl;

typedef struct {
  double dt_adv, dt_ac, vmax, numax, t;
  int32_t n_ac, pad;
  int64_t step;
} sph_step_info;

/* Kernel timing (HIP events on the context stream) for profiling. */
enum { SPH_K_CELLS = 0, SPH_K_CORRECTION = 1, SPH_K_ADVECTION = 2,
       SPH_K_PRESSURE = 3, SPH_K_DENSITY = 4, SPH_K_BUFFER = 5,
       SPH_K_REDUCE = 6, SPH_K_COUNT = 7 };
typedef struct {
  double total_ms;       /* summed kernel durations */
  int64_t launches;
  double bytes;          /* algorithmic HBM bytes summed over launches */
  double particles;      /* particles processed summed over launches */
} sph_kernel_stats;

typedef struct sph_ctx sph_ctx;   /* opaque, library-owned host object */

/* Bytes of device workspace the caller must provide to sph_create.  Returns
 * 0 if the parameters are invalid. */
size_t sph_workspace_size(const sph_params* params, const sph_buffer_desc* bufs,
                          int32_t nbuf);

/* Validates the problem (Sec. 2 parameters, Table 3 buffers), lays out every
 * device array inside `workspace` (device, >= sph_workspace_size bytes,
 * 256-byte aligned, owned by the caller, must outlive the context), uploads
 * the buffer table and each buffer's local cell-linked-list box (Sec. 2.4.1)
 * and records `hip_stream` (a hipStream_t; NULL = null stream).
 * On success *out receives the context. */
sph_status sph_create(const sph_params* params, const sph_buffer_desc* bufs,
                      int32_t nbuf, void* workspace, size_t ws_bytes,
                      void* hip_stream, sph_ctx** out);

/* Releases the host context (never the caller's workspace). */
sph_status sph_destroy(sph_ctx* ctx);

/* Message of the last failure of `ctx` (static string for ctx == NULL). */
const char* sph_last_error(const sph_ctx* ctx);

/* Loads n particles (n <= capacity) from caller device arrays (FP64/uint32,
 * component-major) and sets the id of the next injected particle.  Walls are
 * particles tagged SPH_WALL.  Invalidates the cell list.  Synchronises. */
sph_status sph_set_particles(sph_ctx* ctx, int64_t n, uint64_t next_pid,
                             const sph_particles* src);

/* Number of particle slots currently used (n_total includes particles
 * tagged SPH_DEAD by the last buffer update until the next cell build) and
 * of real (fluid + buffer) particles. */
sph_status sph_get_count(const sph_ctx* ctx, int64_t* n_total, int64_t* n_real);

/* Copies the n_total current particles, in the library's current order,
 * into caller device arrays of at least n_total entries.  Synchronises. */
sph_status sph_get_particles(sph_ctx* ctx, const sph_particles* dst);

/* Sets the step counter and physical time (counter of the inlet noise and
 * argument of the inflow ramp). */
sph_status sph_set_clock(sph_ctx* ctx, int64_t step, double t);

/* Cell-linked-list build (Sec. 2.4.3: rebuilt after deletion every advection
 * step): counting sort of all particles by cell id (ties by particle id),
 * dropping particles tagged SPH_DEAD, and permutation of every field into
 * cell order.  Asynchronous. */
sph_status sph_build_cells(sph_ctx* ctx);

/* Correction matrix B_i, Eq. (equ-B-matrix), with the mirror boundary
 * treatment of Sec. 3.3 at every buffer's open face when obc_mode >= 3
 * (pair sums in the configured precision, inversion in FP64).  Requires
 * sph_build_cells since the last position change (SPH_E_STATE).
 * Asynchronous. */
sph_status sph_correction(sph_ctx* ctx);

/* One advection step of the dual-criteria scheme (Sec. 2.3): time-step
 * reduction, ARD viscous force and k-epsilon update at the advection level,
 * then n_ac acoustic sub-steps (pressure relaxation with the open-boundary
 * compensation of Eq. (eq-pressure-gradient-obc-B-final) and the velocity
 * boundary condition, drift, Riemann continuity).  ctrl may be NULL
 * (adaptive step).  Requires sph_build_cells and sph_correction
 * (SPH_E_STATE).  Synchronises once to read the time-step reduction. */
sph_status sph_step(sph_ctx* ctx, const sph_step_ctrl* ctrl, sph_step_info* out);

/* Bidirectional buffer update (Secs. 2.4.2, 2.4.3, 3.1, 3.2): relabel,
 * inject (append at the end, canonical order by buffer id then parent id,
 * parent recycled by -L_b n_b with the buffer's boundary values) and delete
 * (particle tagged SPH_DEAD, dropped by the next cell build), each decided
 * from one snapshot over the particles of the buffer's local cell list.
 * Requires sph_build_cells since the last update (SPH_E_STATE).  out may be
 * NULL.  Synchronises once to read the counts. */
sph_status sph_buffer_update(sph_ctx* ctx, sph_buffer_counts* out);

/* Decision codes of sph_buffer_update for the current state without
 * applying them (device uint32 [n_total], current order; particles outside
 * every local cell list get SPH_DEC_NONE).  Requires sph_build_cells. */
sph_status sph_buffer_decisions(sph_ctx* ctx, uint32_t* dec);

/* Pair operators at the current state (p and V from rho, B from the last
 * sph_correction) into the FP64 device arrays of `out` (NULL members are
 * skipped; gradv/dk/deps only with turbulence).  Requires sph_correction
 * since the last position change.  Asynchronous. */
sph_status sph_eval_rates(sph_ctx* ctx, const sph_rates* out);

/* Neighbour lists with the FP64 predicate |x_i - x_j|^2 < (2h)^2, j != i,
 * for every particle, as CSR in the current order: row_ptr (device int32
 * [n_total + 1]) and col (device int32 [cap]).  *n_pairs receives the total;
 * SPH_E_CAPACITY if it exceeds cap (row_ptr is still valid).  Requires
 * sph_build_cells since the last position change.  Synchronises. */
sph_status sph_neighbors(sph_ctx* ctx, int32_t* row_ptr, int32_t* col,
                         int64_t cap, int64_t* n_pairs);

/* Kernel timing with HIP events on the context stream. */
sph_status sph_profile_enable(sph_ctx* ctx, int32_t on);
sph_status sph_profile_read(sph_ctx* ctx, int32_t kernel, sph_kernel_stats* out);

/* Directed neighbour pairs evaluated by the neighbour passes since the last
 * call (counted in the continuity pass x 2 + correction + advection).
 * Synchronises. */
sph_status sph_pair_count(sph_ctx* ctx, int64_t* pairs);

#ifdef __cplusplus
}
#endif
#endif
