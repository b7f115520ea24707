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
  int64_t capacity;     /* particle slots: real + wall + reserve for injection, < 2^26 */
  uint64_t seed;        /* counter-based random numbers (inlet noise) */
  double tvf_alpha;     /* transport-velocity shift (Sec. 2.3 names the formulation
                           and cites it without a formula; the form used is
                           dx_i = -tvf_alpha h^2 sum_j 2 V_j grad_i W_ij for fluid
                           particles and, along their open face only,
                           particles of extrapolated-velocity buffers, summed
                           on the start-of-step state and added
                           to the positions at the end of the advection step);
                           0 = off.  The adjoint requires 0. */
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
  double* shift;  /* [3][n] transport-velocity shift (tvf_alpha != 0; 0 for
                     prescribed-velocity buffers and walls); NULL: not written */
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
  int32_t n_ac;
  /* sph_advance: 1 when a particle outgrew the step's neighbour list (the
   * later passes of the step scanned the cell stencil), else 0; sph_step: -1
   * (not known before the next buffer update) */
  int32_t list_outgrown;
  int64_t step;
} sph_step_info;

/* Kernel timing for profiling.  The four neighbour passes (correction,
 * advection, pressure, density: one kernel each) are timed by events that
 * their launch records at the kernel's own start and end; the other entries
 * by a pair of events on the context stream around their launches. */
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

/* Zero-copy access to the particle arrays (Sec. 2.4.3: particles are
 * appended and overwritten in place in preallocated arrays).  Field ids of
 * sph_field_offset and their element types. */
enum { SPH_FIELD_X0 = 0, SPH_FIELD_X1 = 1, SPH_FIELD_X2 = 2, SPH_FIELD_V0 = 3,
       SPH_FIELD_V1 = 4, SPH_FIELD_V2 = 5, SPH_FIELD_RHO = 6, SPH_FIELD_DRHO = 7,
       SPH_FIELD_K = 8, SPH_FIELD_EPS = 9, SPH_FIELD_TAG = 10, SPH_FIELD_PID = 11,
       SPH_FIELD_COUNT = 12 };
enum { SPH_DTYPE_F64 = 0, SPH_DTYPE_F32 = 1, SPH_DTYPE_U32 = 2 };

/* Byte offset, inside the workspace given to sph_create, of the live array
 * of `field` (capacity entries in the library's current particle order) and
 * its element type: FP64 for positions and density; the pair precision
 * (SPH_DTYPE_F64, or SPH_DTYPE_F32 in SPH_FP32_MIXED contexts) for velocity,
 * continuity rate, k and epsilon; uint32 for tags and ids.  The caller may
 * wrap the array in a tensor view and read or write particles in place.  An
 * offset holds until the next call that builds cells, steps, updates the
 * buffers, advances or sets particles (they move the live arrays between two
 * slots): take it again after any of them.  SPH_E_ARG for an unknown field. */
sph_status sph_field_offset(const sph_ctx* ctx, int32_t field, size_t* offset, int32_t* dtype);

/* Declares that the caller has written n_total particles (<= capacity) into
 * the live arrays of sph_field_offset, and sets the id of the next injected
 * particle: the library derives the eddy viscosity C_mu k^2 / epsilon
 * (Table 1) from the k and epsilon written, counts the real particles and
 * invalidates the cell list -- what sph_set_particles does after its copy.
 * SPH_E_ARG (nothing changed) for a count out of range or a buffer particle
 * whose tag names no configured buffer.  Synchronises. */
sph_status sph_set_count(sph_ctx* ctx, int64_t n_total, uint64_t next_pid);

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

/* Step counter, physical time and id of the next injected particle
 * (checkpoint / resume: with sph_get_particles this is the whole state). */
sph_status sph_get_clock(const sph_ctx* ctx, int64_t* step, double* t, uint64_t* next_pid);

/* Cell-linked-list build (Sec. 2.4.3: rebuilt after deletion every advection
 * step): counting sort of all particles by cell id and, inside a cell, by
 * quarter of the cell along x (particles of one quarter keep their relative
 * order in the current arrays), dropping particles tagged SPH_DEAD, and
 * permutation of every field into that order.  Asynchronous. */
sph_status sph_build_cells(sph_ctx* ctx);

/* Correction matrix B_i, Eq. (equ-B-matrix), with the mirror boundary
 * treatment of Sec. 3.3 at every buffer's open face when obc_mode >= 3
 * (pair sums in the configured precision, inversion in FP64).  Also builds
 * the step's neighbour list, which the later passes of the step read: every
 * pair within the cell size or, from 10k particles, within a radius that
 * bounds the pair's relative motion over the coming step (the same list
 * sph_advance builds for the state).  Requires sph_build_cells since the last
 * position change (SPH_E_STATE).  Asynchronous. */
sph_status sph_correction(sph_ctx* ctx);

/* One advection step of the dual-criteria scheme (Sec. 2.3): time-step
 * reduction, ARD viscous force and k-epsilon update at the advection level,
 * then n_ac acoustic sub-steps (pressure relaxation with the open-boundary
 * compensation of Eq. (eq-pressure-gradient-obc-B-final) and the velocity
 * boundary condition, drift, Riemann continuity).  ctrl may be NULL
 * (adaptive step).  Requires sph_build_cells and sph_correction
 * (SPH_E_STATE).  The time-step reduction of a state produced by
 * sph_buffer_update was computed and read back by that update; for any
 * other state sph_step synchronises once to read it. */
sph_status sph_step(sph_ctx* ctx, const sph_step_ctrl* ctrl, sph_step_info* out);

/* Bidirectional buffer update (Secs. 2.4.2, 2.4.3, 3.1, 3.2): relabel,
 * inject (append at the end, canonical order by buffer id then parent id,
 * parent recycled by -L_b n_b with the buffer's boundary values) and delete
 * (particle tagged SPH_DEAD, dropped by the next cell build), each decided
 * from one snapshot over the particles of the buffer's local cell list.
 * Requires sph_build_cells since the last update (SPH_E_STATE).  out may be
 * NULL.  Synchronises once, reading back the counts, the error flags (also
 * those raised by the kernels since the previous read-back) and the
 * time-step reduction of the updated state for the next sph_step. */
sph_status sph_buffer_update(sph_ctx* ctx, sph_buffer_counts* out);

/* sph_buffer_update with an event log and replay, for sensitivity runs.
 * log_by_pid (device uint32 [pid_cap], or NULL): zeroed, then receives the
 * decision code of every particle examined, indexed by particle id.
 * forced_by_pid (device uint32 [pid_cap], or NULL): the decisions to apply
 * instead of the predicates (a log of an earlier run), looked up by
 * particle id for every slot; ids >= pid_cap and non-real particles get
 * SPH_DEC_NONE.  pid_cap must be >= the next particle id when either array
 * is given (SPH_E_ARG).  After an update with injections, the children are
 * the copies of the parents in canonical order (see sph_buffer_update).
 * Synchronises once. */
sph_status sph_buffer_update_ex(sph_ctx* ctx, const uint32_t* forced_by_pid,
                                uint32_t* log_by_pid, int64_t pid_cap,
                                sph_buffer_counts* out);

/* One full advection step as the method advances the flow (Sec. 2.3 with
 * the buffer update of Sec. 2.4 at its end): sph_build_cells,
 * sph_correction, sph_step(ctrl) and sph_buffer_update in one call, with
 * the same results as those calls made in that order.  The cell build and
 * correction of the updated state are enqueued before the update's one
 * read-back (their sizes taken on the device), so on success the state is
 * the updated one already built and corrected: particles tagged SPH_DEAD
 * are dropped and the next sph_advance (or sph_step) starts from it.  (In
 * 3D laminar contexts with the neighbour list, that correction writes the
 * list only and the next step's advection pass forms B from the same walk
 * of the list, bit for bit the B sph_correction forms; sph_eval_rates forms
 * it first when asked for a state left so.)  The
 * first failure returns its status.  On SPH_E_CAPACITY the state is the
 * one a failed sph_buffer_update leaves; on a flag error raised by the step
 * (SPH_E_NUMERIC) it is the updated state and a cell build is required.
 * info and counts may be NULL.  Synchronises once. */
sph_status sph_advance(sph_ctx* ctx, const sph_step_ctrl* ctrl, sph_step_info* info,
                       sph_buffer_counts* counts);

/* Decision codes of sph_buffer_update for the current state without
 * applying them (device uint32 [n_total], current order; particles outside
 * every local cell list get SPH_DEC_NONE).  Requires sph_build_cells. */
sph_status sph_buffer_decisions(sph_ctx* ctx, uint32_t* dec);

/* Pair operators at the current state (p and V from rho, B from the last
 * sph_correction, or formed first for a state left by sph_advance whose B
 * the next step would form) into the FP64 device arrays of `out` (NULL
 * members are skipped; gradv/dk/deps only with turbulence).  Requires
 * sph_correction (or sph_advance) since the last position change.
 * Asynchronous. */
sph_status sph_eval_rates(sph_ctx* ctx, const sph_rates* out);

/* Neighbour lists with the FP64 predicate |x_i - x_j|^2 < (2h)^2, j != i,
 * for every particle, as CSR in the current order: row_ptr (device int32
 * [n_total + 1]) and col (device int32 [cap]).  *n_pairs receives the total;
 * SPH_E_CAPACITY if it exceeds cap (row_ptr is still valid).  Requires
 * sph_build_cells since the last position change.  Synchronises. */
sph_status sph_neighbors(sph_ctx* ctx, int32_t* row_ptr, int32_t* col,
                         int64_t cap, int64_t* n_pairs);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * sph_neighbors with its scratch memory -- the per-particle neighbour counts
 * and the partial sums of their scan -- in a device array of the library
 * instead of the context's workspace.  The array holds
 * SPH_NOALLOC_MAX_PARTICLES + 4096 int32 (16 MiB) per device, from the
 * first sph_create on that device until the process ends; the call
 * allocates nothing (the total is read back through the context's pinned
 * buffer).  SPH_E_ARG when the context holds more than
 * SPH_NOALLOC_MAX_PARTICLES particles.  Every call on one device shares the
 * array: calls that overlap on a device (any context, any stream) race and
 * must be serialised by the caller.  Otherwise as sph_neighbors (same
 * results, same errors).  Synchronises. */
#define SPH_NOALLOC_MAX_PARTICLES 4194304
sph_status sph_neighbors_noalloc(sph_ctx* ctx, int32_t* row_ptr, int32_t* col, int64_t cap,
                                 int64_t* n_pairs);

/* The neighbour pairs that the pair passes of a step visit (Sec. 2.4.1: the
 * cell-linked list; the sums of Eqs. (equ-B-matrix), (eq-discretize-momentum-
 * p-RKGC), (discretize-continuity-equ-riemann) and (eq-discretize-momentum-
 * ARD2) run over them): the candidates of the per-step neighbour list built
 * by sph_correction (the cell stencil when that list is switched off) that
 * pass the passes' own test |x_i - x_j|^2 < (2h)^2, evaluated in the pair
 * precision on cell-relative positions.  CSR in the current order, row_ptr
 * (device int32 [n_total + 1]) and col (device int32 [cap], visiting order);
 * particles that are not real have empty rows.  *n_pairs receives the total;
 * SPH_E_CAPACITY if it exceeds cap (row_ptr is still valid).  Requires
 * sph_correction since the last position change (SPH_E_STATE).  Synchronises. */
sph_status sph_step_pairs(sph_ctx* ctx, int32_t* row_ptr, int32_t* col, int64_t cap,
                          int64_t* n_pairs);

/* Kernel timing with HIP events on the context stream. */
sph_status sph_profile_enable(sph_ctx* ctx, int32_t on);
sph_status sph_profile_read(sph_ctx* ctx, int32_t kernel, sph_kernel_stats* out);

/* Directed neighbour pairs evaluated by the neighbour passes since the last
 * call (counted in the continuity pass x 2 + correction + advection).
 * Synchronises. */
sph_status sph_pair_count(sph_ctx* ctx, int64_t* pairs);

/* ---------------------------------------------------------------------
 * Inlet-profile sensitivity (laminar contexts).  The forward replays run in
 * the context's precision; their sub-step states are kept in FP64 and the
 * reverse sweep is FP64 (with an FP32-mixed context: the FP64 scheme's
 * gradient at the FP32 trajectory).
 *
 * Objectives at the state after sph_step (before the buffer update):
 *   J_Q   = sum over real i with 0 <= n.(x_i - o) < w of m (v_i . n) / w,
 *           the mass flux through a slab (per unit depth in 2D);
 *   J_tau = -(1 / L_w) sum over real i and wall j with |x_i - x_j| < 2h of
 *           m (2 / rho_i) mu f(r_ij) V_j (2 v_i . e),  f = W'(r) / r,
 *           mu = rho0 nu_l: the e-component of the viscous force of the
 *           fluid on the dummy walls (Eq. (eq-discretize-momentum-ARD2) with
 *           the antisymmetric wall velocity) per unit wall length.
 * Parameters: the sine coefficients a_1..a_n of the control buffer's
 * SPH_PROFILE_SINE inlet profile u(s) = 4 u0 s (1 - s) + sum a_m sin(m pi s).
 * --------------------------------------------------------------------- */
typedef struct {
  double slab_origin[3];   /* a point on the slab's upstream plane */
  double slab_normal[3];   /* unit normal n */
  double slab_width;       /* w > 0 */
  double shear_dir[3];     /* unit direction e */
  double wall_length;      /* L_w > 0 */
  int32_t control_buffer;  /* id of the buffer whose coefficients are the parameters */
  int32_t pad;
} sph_objective_desc;

/* Replaces the profile coefficients of buffer `buffer_id` (host array of
 * n_coef <= 16 values; the rest are zeroed).  Synchronises. */
sph_status sph_set_profile_coef(sph_ctx* ctx, int32_t buffer_id, int32_t n_coef,
                                const double* coef);

/* Adds [J_Q, J_tau] of the current state to J (device FP64 [2]).  Slab
 * membership is taken from member_by_pid (device uint8 [pid_cap], a frozen
 * event of a replayed run) when given, else from the positions; it is
 * written to member_out_by_pid (device uint8 [pid_cap], zeroed first) when
 * given.  Laminar contexts only (SPH_E_ARG).  Deterministic.  Asynchronous. */
sph_status sph_objective(sph_ctx* ctx, const sph_objective_desc* obj,
                         const uint8_t* member_by_pid, uint8_t* member_out_by_pid,
                         int64_t pid_cap, double* J);

/* One recorded advection step, as the adjoint replays it. */
typedef struct {
  int64_t step;            /* step counter of the pre-step state */
  double t;                /* time of the pre-step state */
  uint64_t next_pid;       /* next particle id of the pre-step state */
  double dt_adv;           /* the step's advection time step */
  int32_t n_ac;            /* and its acoustic sub-steps */
  int32_t pad;
  const uint32_t* dec_by_pid;    /* device [pid_cap]: the step's buffer decisions */
  const uint8_t* member_by_pid;  /* device [pid_cap]: the step's slab membership */
  int64_t pid_cap;
  double w_flux, w_shear;  /* dL/dJ_Q and dL/dJ_tau of this step's objectives */
} sph_adjoint_ctrl;

/* Device workspace of sph_adjoint_step (or of one step of
 * sph_adjoint_forward / sph_adjoint_reverse) for steps of up to max_nac
 * acoustic sub-steps; 0 when the context cannot run the adjoint
 * (turbulent, or with the transport-velocity shift on). */
size_t sph_adjoint_workspace_size(const sph_ctx* ctx, int32_t max_nac);

/* Discrete adjoint of one advection step followed by its buffer update
 * (decisions, time step and slab membership frozen), on the fixed neighbour
 * sets of the step: the reverse of the continuity, pressure, viscous and
 * correction passes and of the velocity boundary conditions.
 *   pre, n_pre: the state at the start of the step (device FP64 /
 *       uint32 component-major, as sph_get_particles writes it);
 *   lam (device FP64 [8][pid_cap], rows x0 x1 x2 v0 v1 v2 rho drho, by
 *       particle id): on entry the cotangent of the state after the step's
 *       buffer update; on return that of the state at the start of the step
 *       (entries of particles created by the update are zeroed);
 *   grad (device FP64 [16]): receives += dL/da through the step.
 * The replay overwrites the context's particle state.  Synchronises. */
sph_status sph_adjoint_step(sph_ctx* ctx, const sph_particles* pre, int64_t n_pre,
                            const sph_objective_desc* obj, const sph_adjoint_ctrl* ctl,
                            double* lam, double* grad, void* adj_ws, size_t adj_bytes);

/* The two halves of sph_adjoint_step, for a reverse sweep that does not
 * replay each step a second time (the checkpointed recomputation of a
 * segment runs sph_adjoint_forward, one workspace per step, and the reverse
 * then walks the workspaces back).
 *
 * sph_adjoint_forward: the recorded step (same ctl as sph_adjoint_step)
 * from the context's current state, which must be the step's start state
 * (its next particle id must equal ctl->next_pid: SPH_E_STATE): cell build,
 * correction with the neighbour list, the step with every sub-step state
 * kept in adj_ws, and the replayed buffer update.  adj_ws also keeps the
 * step's cell build, list, correction matrices and update data, so that the
 * reverse does not read the context's state.  *n_step receives the step's
 * particle slots.  Leaves the context at the state after the update.
 * Synchronises once (the replayed update's read-back of its counts).
 *
 * sph_adjoint_reverse: the reverse sweep of sph_adjoint_step from a
 * workspace filled by sph_adjoint_forward (and n_step from that call); lam
 * and grad as in sph_adjoint_step.  Reads no particle state of the context.
 * Synchronises. */
sph_status sph_adjoint_forward(sph_ctx* ctx, const sph_adjoint_ctrl* ctl, void* adj_ws,
                               size_t adj_bytes, int64_t* n_step);
sph_status sph_adjoint_reverse(sph_ctx* ctx, const sph_objective_desc* obj,
                               const sph_adjoint_ctrl* ctl, int64_t n_step, double* lam,
                               double* grad, void* adj_ws, size_t adj_bytes);

#ifdef __cplusplus
}
#endif
#endif
