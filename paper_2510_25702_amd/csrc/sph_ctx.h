// Host-side context of the gfx950 SPH pipeline and the launcher interface
// between the C ABI (sph_abi.hip) and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <string>
#include <vector>

#include "../../include/sph.h"
#include "sph_device.h"

namespace sphx {

// Most workgroups of the post-update reduction (each leaves its maxima in
// the pinned read-back buffer for the host to combine).
constexpr int kPostBlocks = 1024;

// Two-slot ("ping-pong") device array: cur() is the live copy.
template <typename P>
struct Slot2 {
  P* a[2] = {nullptr, nullptr};
  int cur = 0;
  P* live() const { return a[cur]; }
  P* other() const { return a[cur ^ 1]; }
  void flip() { cur ^= 1; }
};

// Every per-particle field, as raw device pointers inside the workspace.  The
// pair-precision arrays are typed void* here and cast by the launchers.
struct Fields {
  Slot2<double> x[3];      // master positions (FP64)
  Slot2<void> xr[3];       // cell-relative positions (pair precision)
  Slot2<void> v[3];        // velocity (pair precision)
  Slot2<double> rho;       // density (FP64)
  Slot2<void> drho;        // last continuity rate
  Slot2<void> k, eps, nut; // RANS
  Slot2<uint32_t> tag, pid;
  Slot2<void> p, vol;      // effective pressure and volume, per sub-step
  void* B[6];              // symmetric correction matrix (pair precision)
  void* anu[3];            // viscous acceleration of the advection step
  int32_t* cell;           // build-time cell id per particle
  // per-step neighbour list (radius = cell size), built with B
  uint32_t* nbr;           // [K/C][cap][C] j | stencil offset code << 27 (nbr_index)
  int32_t* ncnt;           // [cap] entries of particle i
  void* xrb[3];            // cell-relative positions at the list build
  int nbr_k;               // K
  // j-side records of the pressure / continuity passes (16-byte vectors of T)
  void* prec[3];           // position, p, volume (negative: wall), B
  void* drec[2];           // position, velocity, p, volume (negative: wall)
  void* arec[3];           // position, velocity, volume (negative: wall), RANS fields
  void* shift[3];          // transport-velocity shift of the step (NULL: off)
  // relative-motion list radius (builds launched by sph_advance): the mean
  // velocity of each cell's moving particles and each particle's allowed
  // deviation from drifting with it over the step
  void* cell_u[3];         // [ncell] (pair precision)
  float* lskin;            // [cap]
  float* xr32[3];          // [cap] FP32 copies of xr for the FP64 list scan (FP64 only)
};

struct Scratch {
  int32_t* key;            // [cap] cell id of a particle (-1: dropped)
  int32_t* slot;           // [cap] rank inside the cell (atomic)
  int32_t* perm;           // [cap] sorted position -> source index
  int32_t* count;          // [ncell] particles per cell
  int32_t* cell_start;     // [ncell + 1]
  int32_t* cell_q;         // [4 ncell] starts of the x quarters 1-3 of each cell
  int32_t* block_sums;     // scan partials
  uint32_t* dec;           // [cap] buffer decisions
  int32_t* cand_cells;     // candidate cells of the buffer update
  int32_t n_cand_cells;
  uint64_t* inj_key;       // [kMaxInject]
  int32_t* inj_idx;        // [kMaxInject]
  int32_t* counters;       // [4 * 256 + 16] per-buffer counts + misc
  uint32_t* flags;         // [1] error flags
  uint32_t* stale;         // [2] neighbour list outgrown (by sub-step parity)
  int32_t* nstate;         // [4] next build's sizes after an update: n_in, n_out, skip
  double* lrad;            // [4] Δt_ad of the coming step (0: unknown), list mode of the build
  double* red;             // reduction partials
  long long* pairs;        // [1] pair counter
  uint64_t* next_pid;      // [1]
  BufDev* bufs;            // [kMaxBuf]
  int32_t* bidx;           // [256] buffer index of an id (-1: none)
};

struct Profile {
  bool on = false;
  struct Rec { int kernel; hipEvent_t a, b; double bytes, particles; };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  double total_ms[SPH_K_COUNT] = {0};
  long long launches[SPH_K_COUNT] = {0};
  double bytes[SPH_K_COUNT] = {0};
  double particles[SPH_K_COUNT] = {0};
  hipEvent_t ext_a = nullptr, ext_b = nullptr;   // for the next launch_pass to record
  int open = -1;                                   // section being timed (-1: none)
};

}  // namespace sphx

struct sph_ctx {
  sph_params P;
  std::vector<sph_buffer_desc> bufs_h;
  std::vector<sphx::BufDev> bufdev_h;
  int nbuf = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  sphx::GridDev grid;
  sphx::Fields F;
  sphx::Scratch S;
  int64_t cap = 0;
  int64_t n_total = 0;       // used slots (incl. particles tagged dead)
  int64_t n_alive = 0;       // slots that survive the next cell build
  int64_t n_real = 0;
  uint64_t next_pid = 0;
  int64_t step = 0;
  double t = 0.0;
  bool cells_valid = false;  // cell list matches the current arrays
  bool moved = false;        // positions changed since the cell build
  bool B_valid = false;
  bool need_pv0 = false;
  int pv_half = 0;
  uint32_t* pinned = nullptr;   // host staging (pinned)
  int32_t* pinned_dev = nullptr;  // its device address (the post-update reduction writes there)
  int team_override = 0;        // lanes per particle of the neighbour passes (0: auto)
  int corr_override = 0;        // lanes per particle of the correction pass (0: auto)
  bool use_nbr = true;          // neighbour passes read the per-step list
  int tight_list = -1;          // relative-motion list radius: 1 on, 0 off, -1 by size
  bool B_pending = false;       // B of the current state is formed by the next advection pass
  bool last_outgrown = false;   // the last updated step's list was outgrown
  bool nbr_valid = false;       // the list matches the current cell build
  int substep = 0;              // acoustic sub-step being launched
  bool red_valid = false;       // red_v2 / red_nut hold the reduction of the current state
  double red_v2 = 0.0, red_nut = 0.0;
  int post_blocks = 0;            // workgroups of the last post-update reduction
  hipEvent_t rb_event = nullptr;  // marks the buffer update's read-back copy
  std::string err;
  sphx::Profile prof;
};

namespace sphx {

// Launchers implemented in the kernel translation units.  Each enqueues on
// ctx->stream and returns the HIP error of the launch.
hipError_t launch_zero_i32(sph_ctx* c, int32_t* p, int64_t n);
hipError_t launch_set_particles(sph_ctx* c, int64_t n, const sph_particles* src);
hipError_t launch_get_particles(sph_ctx* c, const sph_particles* dst);
// eddy viscosity C_mu k^2 / epsilon of the n live particles (after the
// caller wrote k and epsilon in place)
hipError_t launch_derive_nut(sph_ctx* c, int64_t n);
// With ns (device {n_in, n_out, skip}, written by the post-update reduction)
// the sizes are read on the device and n_in / n_grid are upper bounds.
// keys_done: that reduction also computed the cell keys, slots and counts
// (launch_reduce with keys), so the build starts at the scan.
hipError_t launch_build_cells(sph_ctx* c, int64_t n_in, int64_t n_out,
                              const int32_t* ns = nullptr, bool keys_done = false);
// tight: the list takes the relative-motion radius (the coming step's Δt_ad
// on the device, from launch_list_dt); otherwise the cell size
// moment false (3D laminar list passes): only the list; the step's advection
// pass forms B (B_pending until then, launch_moment forms it on demand)
hipError_t launch_correction(sph_ctx* c, const int32_t* ns = nullptr, int64_t n_grid = 0,
                             bool tight = false, bool moment = true);
hipError_t launch_moment(sph_ctx* c);
// the coming step's Δt_ad, as the host forms it, into S.lrad[0]: from the
// post-update reduction's maxima (a build launched before the host has
// them), or with fresh a reduction of the current state first
hipError_t launch_list_dt(sph_ctx* c, bool fresh = false);
// time-step reduction (max |v|^2, max nu_t, flags) into S.red[0..2], and
// into host memory when out_host3 is given; after_update also covers the
// particles the last buffer update appended
// keys (after_update only): also the cell keys, slots and counts of the
// updated arrays for the next build (launch_build_cells with keys_done)
hipError_t launch_reduce(sph_ctx* c, double* out_host3, bool after_update = false,
                         bool keys = false);
// Adds the transport-velocity shift of the advection pass to the positions
// of fluid particles (the end of the advection step).
hipError_t launch_shift_apply(sph_ctx* c);
hipError_t launch_advection(sph_ctx* c, double dt_adv, double dt_sub, bool rates_only,
                            const sph_rates* out);
hipError_t launch_pressure(sph_ctx* c, double dt, bool rates_only, const sph_rates* out);
hipError_t launch_density(sph_ctx* c, double dt, bool last, bool rates_only,
                          const sph_rates* out);
hipError_t launch_prepare_pv(sph_ctx* c, const sph_rates* out);
hipError_t launch_buffer_decide(sph_ctx* c, bool dry, uint32_t* dec_out, uint32_t* log = nullptr,
                                int64_t pid_cap = 0);
hipError_t launch_buffer_forced(sph_ctx* c, const uint32_t* forced, uint32_t* log, int64_t pid_cap);
hipError_t launch_buffer_inject(sph_ctx* c);
hipError_t launch_buffer_undo(sph_ctx* c, bool all_slots);
hipError_t launch_neighbors(sph_ctx* c, int32_t* row_ptr, int32_t* col, int64_t cap,
                            int64_t* n_pairs);
hipError_t launch_export_B(sph_ctx* c, double* B);
// exclusive scan of n counts into out[0..n] (out[n] = total); the partial
// sums of up to 4096 tiles in the workspace, or in `part`
hipError_t launch_scan_excl(sph_ctx* c, const int32_t* in, int n, int32_t* out);
hipError_t launch_scan_excl_part(sph_ctx* c, const int32_t* in, int n, int32_t* out,
                                 int32_t* part);
// The library's own device array of sph_neighbors_noalloc: its address on
// `device` (the current device), taken once per device.
hipError_t noalloc_scratch_init(int device);
// sph_neighbors with its scratch in that array; synchronises
hipError_t launch_neighbors_noalloc(sph_ctx* c, int32_t* row_ptr, int32_t* col, int64_t cap,
                                    int64_t* n_pairs);
// the pairs the pair passes visit (CSR in the current order); synchronises
// once to read the total
hipError_t launch_walk_pairs(sph_ctx* c, int32_t* row_ptr, int32_t* col, int64_t cap,
                             int64_t* n_pairs);

// sensitivity (k_adjoint.hip)
size_t adjoint_ws_bytes(const sph_ctx* c, int max_nac);
hipError_t launch_objective(sph_ctx* c, const sph_objective_desc* obj, const uint8_t* member_in,
                            uint8_t* member_out, int64_t pid_cap, double* J);
hipError_t adjoint_snap_start(sph_ctx* c, char* ws, int N);
hipError_t adjoint_snap_advection(sph_ctx* c, char* ws, int N);
hipError_t adjoint_snap_pressure(sph_ctx* c, char* ws, int N, int s);
hipError_t adjoint_snap_density(sph_ctx* c, char* ws, int N, int s);
hipError_t adjoint_keep_step(sph_ctx* c, char* ws, int N, int n_step);
hipError_t adjoint_reverse_launch(sph_ctx* c, char* ws, const sph_objective_desc* obj,
                                  const sph_adjoint_ctrl* ctl, int n, double* lam, double* grad);

size_t pair_bytes(const sph_ctx* c);
void prof_begin(sph_ctx* c, int kernel, double bytes, double particles);
void prof_end(sph_ctx* c);

}  // namespace sphx
