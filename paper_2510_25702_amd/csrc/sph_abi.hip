// C ABI of the gfx950 SPH pipeline (declared in include/sph.h): parameter
// validation, workspace layout, call sequencing, time-step selection and
// kernel timing.  All device memory comes from the caller's workspace.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

#include "sph_ctx.h"

using namespace sphx;

namespace {

const char* kNoCtx = "sph: null context";

sph_status fail(sph_ctx* c, sph_status s, const char* msg) {
  if (c) c->err = msg;
  return s;
}

sph_status hip_fail(sph_ctx* c, hipError_t e, const char* where) {
  if (c) {
    c->err = std::string(where) + ": " + hipGetErrorString(e);
  }
  return SPH_E_HIP;
}

#define HIPCHK(c, expr, where)                     \
  do {                                             \
    hipError_t e_ = (expr);                        \
    if (e_ != hipSuccess) return hip_fail(c, e_, where); \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
  size_t total = 0;
  size_t take(size_t bytes) {
    size_t off = total;
    total += align256(bytes ? bytes : 1);
    return off;
  }
};

const char* validate(const sph_params* P, const sph_buffer_desc* B, int32_t nbuf) {
  if (!P) return "params is NULL";
  if (P->dim != 2 && P->dim != 3) return "dim must be 2 or 3";
  if (P->precision != SPH_FP64 && P->precision != SPH_FP32_MIXED) return "bad precision";
  if (P->turbulence != 0 && P->turbulence != 1) return "turbulence must be 0 or 1";
  if (P->obc_mode < 1 || P->obc_mode > 4) return "obc_mode must be 1..4";
  if (!(P->tvf_alpha >= 0.0 && P->tvf_alpha <= 1.0)) return "tvf_alpha must be in [0, 1]";
  if (!(P->dp > 0) || !(P->h > 0) || !(P->rho0 > 0) || !(P->c0 > 0)) return "dp, h, rho0, c0 must be > 0";
  if (!(P->nu_l >= 0)) return "nu_l must be >= 0";
  if (!(P->cell_size >= 2.0 * P->h)) return "cell_size must be >= 2h";
  if (!(P->cfl_adv > 0) || !(P->cfl_ac > 0) || !(P->u_ref > 0)) return "cfl_adv, cfl_ac, u_ref must be > 0";
  if (P->turbulence && (!(P->k_floor > 0) || !(P->eps_floor > 0))) return "k/eps floors must be > 0";
  if (P->capacity <= 0 || P->capacity >= ((int64_t)1 << kNbrIdxBits)) return "capacity out of range";
  for (int k = 0; k < P->dim; ++k)
    if (!(P->hi[k] - P->lo[k] >= 3.0 * P->cell_size)) return "grid must span >= 3 cells per axis";
  int64_t ncell = 1;
  for (int k = 0; k < P->dim; ++k) {
    double nk = std::ceil((P->hi[k] - P->lo[k]) / P->cell_size);
    if (!(nk < 1e8)) return "grid too large";
    ncell *= (int64_t)nk;
  }
  if (ncell > 16 * 1024 * 1024) return "more than 16M cells";
  if (nbuf < 0 || nbuf > SPH_MAX_BUFFERS) return "nbuf out of range";
  if (nbuf > 0 && !B) return "buffers is NULL";
  for (int q = 0; q < nbuf; ++q) {
    const sph_buffer_desc& b = B[q];
    if (b.id < 1 || b.id > 255) return "buffer id must be 1..255";
    if (q > 0 && b.id <= B[q - 1].id) return "buffer ids must be unique and ascending";
    if (!(b.length > 0) || !(b.half_width[0] > 0) || !(b.fringe >= 0)) return "bad buffer box";
    if (P->dim == 3 && !(b.half_width[1] > 0)) return "bad 3D buffer box";
    if (b.n_coef < 0 || b.n_coef > 16) return "n_coef must be 0..16";
    if (b.vel_mode < 0 || b.vel_mode > 1 || b.p_mode < 0 || b.p_mode > 2 ||
        b.turb_mode < 0 || b.turb_mode > 1 || b.profile < 0 || b.profile > 2)
      return "bad buffer mode";
    if (P->turbulence && b.turb_mode == SPH_TURB_FREESTREAM && !(b.eps_bc > 0))
      return "free-stream eps must be > 0";
  }
  return nullptr;
}

void grid_of(const sph_params* P, GridDev* g) {
  for (int k = 0; k < 3; ++k) {
    g->lo[k] = P->lo[k];
    g->n[k] = k < P->dim ? (int32_t)std::ceil((P->hi[k] - P->lo[k]) / P->cell_size) : 1;
  }
  g->cs = P->cell_size;
  g->ncell = g->n[0] * g->n[1] * g->n[2];
}

// Local cell-linked-list box of a buffer (Sec. 2.4.1): the cells of the
// global grid covering the box widened by one cell, FP64, no contraction.
#pragma clang fp contract(off)
void lcll_box(const sph_params* P, const GridDev& g, const sph_buffer_desc& b, int32_t lo_c[3],
              int32_t hi_c[3]) {
  double cs = P->cell_size, m = cs;
  double y0s[2] = {-m, b.length + b.fringe + m};
  double y1s[2] = {-b.half_width[0] - m, b.half_width[0] + m};
  double y2s[2] = {0.0, 0.0};
  if (P->dim == 3) {
    y2s[0] = -b.half_width[1] - m;
    y2s[1] = b.half_width[1] + m;
  }
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int a = 0; a < 2; ++a)
    for (int c = 0; c < 2; ++c)
      for (int d = 0; d < 2; ++d)
        for (int k = 0; k < 3; ++k) {
          double gk = b.origin[k] + ((y0s[a] * b.frame[k] + y1s[c] * b.frame[3 + k]) +
                                     y2s[d] * b.frame[6 + k]);
          if (gk < lo[k]) lo[k] = gk;
          if (gk > hi[k]) hi[k] = gk;
        }
  for (int k = 0; k < 3; ++k) {
    if (k >= P->dim) {
      lo_c[k] = hi_c[k] = 0;
      continue;
    }
    int64_t a = (int64_t)std::floor((lo[k] - P->lo[k]) / cs);
    int64_t c = (int64_t)std::floor((hi[k] - P->lo[k]) / cs);
    if (a < 0) a = 0;
    if (c > g.n[k] - 1) c = g.n[k] - 1;
    lo_c[k] = (int32_t)a;
    hi_c[k] = (int32_t)c;
  }
}
#pragma clang fp contract(on)

std::vector<int32_t> candidate_cells(const sph_params* P, const GridDev& g,
                                     const sph_buffer_desc* B, int nbuf) {
  std::vector<char> mark((size_t)g.ncell, 0);
  for (int q = 0; q < nbuf; ++q) {
    int32_t lo[3], hi[3];
    lcll_box(P, g, B[q], lo, hi);
    for (int k = 0; k < P->dim; ++k) {   // one more cell for the drift since the build
      lo[k] = std::max(lo[k] - 1, 1);
      hi[k] = std::min(hi[k] + 1, g.n[k] - 2);
    }
    for (int z = lo[2]; z <= hi[2]; ++z)
      for (int y = lo[1]; y <= hi[1]; ++y)
        for (int x = lo[0]; x <= hi[0]; ++x) mark[((size_t)z * g.n[1] + y) * g.n[0] + x] = 1;
  }
  std::vector<int32_t> out;
  for (int32_t c = 0; c < g.ncell; ++c)
    if (mark[c]) out.push_back(c);
  return out;
}

struct Plan {
  Layout L;
  size_t off_x[3][2], off_xr[3][2], off_v[3][2], off_rho[2], off_drho[2], off_k[2], off_eps[2],
      off_nut[2], off_tag[2], off_pid[2], off_p[2], off_vol[2], off_B[6], off_anu[3], off_cell,
      off_key, off_slot, off_perm, off_dec, off_count, off_cstart, off_bsums, off_cand,
      off_injk, off_inji, off_counters, off_flags, off_red, off_pairs, off_npid, off_bufs,
      off_bidx, off_nbr, off_ncnt, off_xrb[3], off_stale, off_prec[3], off_drec[2], off_arec[3], off_nstate,
      off_shift[3], off_cellu[3], off_lskin, off_lrad, off_cellq, off_xr32[3];
  int n_cand;
};

void make_plan(const sph_params* P, const sph_buffer_desc* B, int nbuf, Plan* pl) {
  Layout& L = pl->L;
  const size_t C = (size_t)P->capacity;
  const size_t sT = P->precision == SPH_FP64 ? 8 : 4;
  GridDev g;
  grid_of(P, &g);
  for (int k = 0; k < 3; ++k)
    for (int s = 0; s < 2; ++s) {
      pl->off_x[k][s] = L.take(C * 8);
      pl->off_xr[k][s] = L.take(C * sT);
      pl->off_v[k][s] = L.take(C * sT);
    }
  for (int s = 0; s < 2; ++s) {
    pl->off_rho[s] = L.take(C * 8);
    pl->off_drho[s] = L.take(C * sT);
    pl->off_k[s] = L.take(C * sT);
    pl->off_eps[s] = L.take(C * sT);
    pl->off_nut[s] = L.take(C * sT);
    pl->off_tag[s] = L.take(C * 4);
    pl->off_pid[s] = L.take(C * 4);
    pl->off_p[s] = L.take(C * sT);
    pl->off_vol[s] = L.take(C * sT);
  }
  for (int k = 0; k < 6; ++k) pl->off_B[k] = L.take(C * sT);
  for (int k = 0; k < 3; ++k) pl->off_anu[k] = L.take(C * sT);
  pl->off_cell = L.take(C * 4);
  pl->off_nbr = L.take(C * 4 * (size_t)(P->dim == 2 ? kNbrMax2 : kNbrMax3));
  pl->off_ncnt = L.take(C * 4);
  for (int k = 0; k < 3; ++k) pl->off_xrb[k] = L.take(C * sT);
  for (int k = 0; k < 3; ++k) pl->off_prec[k] = L.take((P->dim == 3 || k < 2) ? C * 4 * sT : 0);
  for (int k = 0; k < 2; ++k) pl->off_drec[k] = L.take(C * 4 * sT);
  for (int k = 0; k < 3; ++k) pl->off_arec[k] = L.take((P->dim == 3 || k < 2) ? C * 4 * sT : 0);
  for (int k = 0; k < 3; ++k) pl->off_shift[k] = L.take(P->tvf_alpha != 0.0 ? C * sT : 0);
  pl->off_key = L.take(C * 4);
  pl->off_slot = L.take(C * 4);
  pl->off_perm = L.take(C * 4);
  pl->off_dec = L.take(C * 4);
  for (int k = 0; k < 3; ++k) pl->off_cellu[k] = L.take((size_t)g.ncell * sT);
  pl->off_lskin = L.take(C * 4);
  const bool x32 = P->precision == SPH_FP64 && P->dim == 3;   // the 3D FP64 list scan's
  for (int k = 0; k < 3; ++k) pl->off_xr32[k] = L.take(x32 ? C * 4 : 0);
  pl->off_lrad = L.take(32);
  pl->off_count = L.take((size_t)g.ncell * 4);
  pl->off_cstart = L.take(((size_t)g.ncell + 1) * 4);
  pl->off_cellq = L.take((size_t)g.ncell * 16);
  pl->off_bsums = L.take(4096 * 4);
  std::vector<int32_t> cand = candidate_cells(P, g, B, nbuf);
  pl->n_cand = (int)cand.size();
  pl->off_cand = L.take(cand.size() * 4);
  pl->off_injk = L.take((size_t)kMaxInject * 8);
  pl->off_inji = L.take((size_t)kMaxInject * 4);
  pl->off_counters = L.take(1040 * 4);
  pl->off_flags = L.take(4);
  pl->off_stale = L.take(8);
  pl->off_nstate = L.take(16);
  pl->off_red = L.take((C / 256 + 8) * 2 * 8 + 64);
  pl->off_pairs = L.take(sizeof(long long) * kPairShards * kPairShardStride);
  pl->off_npid = L.take(8);
  pl->off_bufs = L.take(sizeof(BufDev) * kMaxBuf);
  pl->off_bidx = L.take(256 * 4);
}

// ---------------------------------------------------------------------------
// kernel timing
// ---------------------------------------------------------------------------
hipEvent_t take_event(sph_ctx* c) {
  if (!c->prof.pool.empty()) {
    hipEvent_t e = c->prof.pool.back();
    c->prof.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void resolve_events(sph_ctx* c) {
  std::vector<Profile::Rec> keep;
  for (auto& r : c->prof.pending) {
    if (hipEventQuery(r.b) != hipSuccess) {
      keep.push_back(r);
      continue;
    }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      c->prof.total_ms[r.kernel] += ms;
      c->prof.launches[r.kernel] += 1;
      c->prof.bytes[r.kernel] += r.bytes;
      c->prof.particles[r.kernel] += r.particles;
    }
    c->prof.pool.push_back(r.a);
    c->prof.pool.push_back(r.b);
  }
  c->prof.pending.swap(keep);
}


}  // namespace

namespace sphx {

// Algorithmic bytes per particle of one launch of each neighbour kernel:
// every input field of the particle read once plus every output written once.
double kernel_bytes_per_particle(const sph_ctx* c, int kernel) {
  const double sT = c->P.precision == SPH_FP64 ? 8.0 : 4.0;
  const double d = c->P.dim;
  const double nB = d == 2 ? 3 : 6;
  const bool turb = c->P.turbulence != 0;
  switch (kernel) {
    case SPH_K_CORRECTION:  // xr, vol, tag, cell -> B
      return d * sT + sT + 4 + 4 + nB * sT;
    case SPH_K_ADVECTION:   // xr, v, vol, rho, drho, tag, cell -> anu(3), rho, p, vol
      return d * sT + d * sT + sT + 8 + sT + 4 + 4 + 3 * sT + 8 + 2 * sT +
             (turb ? nB * sT + 3 * sT + 3 * sT : 0.0);
    case SPH_K_PRESSURE:    // xr, p, vol, B, rho, v, anu, tag, cell, x(3), pid -> v, x(3), xr(3)
      return d * sT + 2 * sT + nB * sT + 8 + d * sT + 3 * sT + 4 + 4 + 3 * 8 + 4 + d * sT +
             3 * 8 + 3 * sT;
    case SPH_K_DENSITY:     // xr, v, p, vol, tag, cell, rho -> drho, rho, p, vol
      return d * sT + d * sT + 2 * sT + 4 + 4 + 8 + sT + 8 + 2 * sT + (turb ? sT : 0.0);
    case SPH_K_CELLS:       // keys, scatter, gather of every field (read + write)
      return 3 * 8 + 4 + 8 + 8 + 4 + 2 * (4 + 4) +
             2 * (3 * 8 + 3 * sT + 8 + sT + 4 + 4 + (turb ? 3 * sT : 0.0)) + 3 * sT + sT + 4;
    default:
      return 0.0;
  }
}

// The neighbour passes launch one kernel each: their events are recorded by
// that launch itself, at the kernel's start and end (launch_pass), so the
// duration holds no marker overhead.  Other sections are bracketed by a
// pair of events on the stream.
void prof_begin(sph_ctx* c, int kernel, double bytes, double particles) {
  c->prof.open = -1;
  c->prof.ext_a = c->prof.ext_b = nullptr;
  if (!c->prof.on) return;
  hipEvent_t a = take_event(c), b = take_event(c);
  if (!a || !b) return;
  const bool ext = kernel == SPH_K_CORRECTION || kernel == SPH_K_ADVECTION ||
                   kernel == SPH_K_PRESSURE || kernel == SPH_K_DENSITY;
  if (ext) {
    c->prof.ext_a = a;
    c->prof.ext_b = b;
  } else if (hipEventRecord(a, c->stream) != hipSuccess) {
    return;
  }
  c->prof.pending.push_back({kernel, a, b, bytes, particles});
  c->prof.open = kernel;
}

void prof_end(sph_ctx* c) {
  if (!c->prof.on || c->prof.open < 0 || c->prof.pending.empty()) return;
  const Profile::Rec& r = c->prof.pending.back();
  if (c->prof.ext_a) {   // the section launched nothing: an empty interval
    (void)hipEventRecord(r.a, c->stream);
    (void)hipEventRecord(r.b, c->stream);
  } else if (!(r.kernel == SPH_K_CORRECTION || r.kernel == SPH_K_ADVECTION ||
               r.kernel == SPH_K_PRESSURE || r.kernel == SPH_K_DENSITY)) {
    (void)hipEventRecord(r.b, c->stream);
  }
  c->prof.ext_a = c->prof.ext_b = nullptr;
  c->prof.open = -1;
}

}  // namespace sphx

namespace {

// Below this many particles the relative-motion radius's two extra launches
// per step cost about what its shorter list saves: measured per step (FP32-
// mixed / FP64) with and without it, the 5.2k-particle channel 0.147 / 0.145
// against 0.148 / 0.143 ms, the 57.6k U-channel 0.230 / 0.281 against 0.240
// / 0.293, the 138k adjoint channel 0.278 against 0.293, the 160k jet 0.339
// against 0.359.
constexpr int64_t kTightMinN = 10000;

// Whether the list built for the current state takes the relative-motion
// radius (sph_advance and sph_correction decide alike).
bool list_tight(const sph_ctx* c) {
  if (!c->use_nbr) return false;
  return c->tight_list > 0 || (c->tight_list < 0 && c->n_total >= kTightMinN);
}

sph_status check_flags(sph_ctx* c, uint32_t f) {
  if (f & kFlagCapacity) return fail(c, SPH_E_CAPACITY, "particle capacity / injection limit exceeded");
  if (f & kFlagOutOfGrid) return fail(c, SPH_E_NUMERIC, "particle outside the cell grid");
  if (f & kFlagSkin) return fail(c, SPH_E_NUMERIC, "particle moved beyond the cell skin in one step");
  if (f & kFlagCountMismatch) return fail(c, SPH_E_NUMERIC, "cell count mismatch");
  if (f & kFlagNonFinite) return fail(c, SPH_E_NUMERIC, "non-finite value");
  return SPH_OK;
}

void profile_launch(sph_ctx* c, int kernel) {
  if (!c->prof.on) return;
  double n = (double)c->n_total;
  prof_begin(c, kernel, n * kernel_bytes_per_particle(c, kernel), n);
}

// The buffer update: decisions (predicates, or a replayed log) applied with
// their tag changes, injection, the post-update reduction and one read-back.
// With prelaunch the cell build and correction of the updated state are
// enqueued before the host waits for the read-back, their sizes read on the
// device (written by the reduction), so the GPU has work while the host
// takes the counts and returns; a failed injection turns them into no-ops.
sph_status buffer_update(sph_ctx* c, const uint32_t* forced_by_pid, uint32_t* log_by_pid,
                         int64_t pid_cap, sph_buffer_counts* out, bool prelaunch) {
  if (!c) return SPH_E_ARG;
  if (!c->cells_valid) return fail(c, SPH_E_STATE, "sph_buffer_update needs sph_build_cells first");
  if ((forced_by_pid || log_by_pid) && pid_cap < (int64_t)c->next_pid)
    return fail(c, SPH_E_ARG, "pid_cap must cover every particle id (>= next_pid)");
  profile_launch(c, SPH_K_BUFFER);
  // the counters were cleared by the cell build (the call requires one since
  // the last update; a failed update clears them itself)
  hipError_t e = hipSuccess;
  if (log_by_pid) e = launch_zero_i32(c, (int32_t*)log_by_pid, pid_cap);
  if (e == hipSuccess) {
    if (forced_by_pid) e = launch_buffer_forced(c, forced_by_pid, log_by_pid, pid_cap);
    else e = launch_buffer_decide(c, false, nullptr, log_by_pid, pid_cap);
  }
  if (e == hipSuccess) e = launch_buffer_inject(c);
  prof_end(c);
  if (e != hipSuccess) return hip_fail(c, e, "buffer_update");
  char* hb = (char*)c->pinned;
  c->red_valid = false;
  // the reduction writes the counts, flags, next id and maxima into the
  // pinned buffer itself: the event after it is the read-back
  HIPCHK(c, launch_reduce(c, nullptr, true, prelaunch), "reduce");
  HIPCHK(c, hipEventRecord(c->rb_event, c->stream), "read-back event");
  const Fields saved = c->F;
  const bool nbr_saved = c->nbr_valid;
  bool pre = false;
  if (prelaunch) {
    const int64_t n_max = std::min<int64_t>(c->cap, c->n_total + kMaxInject);
    // the coming step's Δt_ad for the list radius, from the maxima just reduced
    const bool tight = list_tight(c);
    e = tight ? launch_list_dt(c) : hipSuccess;
    profile_launch(c, SPH_K_CELLS);
    if (e == hipSuccess)
      e = launch_build_cells(c, n_max, n_max, c->S.nstate, true);   // keys came with the reduction
    prof_end(c);
    if (e == hipSuccess) {
      profile_launch(c, SPH_K_CORRECTION);
      // the list only: the step that follows forms B in its advection pass
      e = launch_correction(c, c->S.nstate, n_max, tight, false);
      prof_end(c);
    }
    if (e != hipSuccess) {
      (void)hipStreamSynchronize(c->stream);
      c->F = saved;
      c->cells_valid = c->B_valid = c->nbr_valid = false;
      return hip_fail(c, e, "cell build");
    }
    pre = true;
  }
  HIPCHK(c, hipEventSynchronize(c->rb_event), "buffer sync");
  if (c->prof.on) resolve_events(c);
  const int32_t* cnt = (const int32_t*)hb;
  uint32_t flags = (uint32_t)cnt[1032];
  c->last_outgrown = cnt[1035] != 0;
  if (flags & kFlagCapacity) {
    // nothing was injected (and the prelaunched kernels returned at once):
    // undo the tag changes the decisions applied, clear the flag and the
    // counters so that the state stays usable
    uint32_t zero = 0;
    if (pre) {
      (void)hipStreamSynchronize(c->stream);
      c->F = saved;
      c->nbr_valid = nbr_saved;
    }
    (void)launch_buffer_undo(c, forced_by_pid != nullptr);
    (void)launch_zero_i32(c, c->S.counters, 1040);
    (void)hipMemcpyAsync(c->S.flags, &zero, 4, hipMemcpyHostToDevice, c->stream);
    (void)hipStreamSynchronize(c->stream);
    return fail(c, SPH_E_CAPACITY, (flags & kFlagInjectOverflow)
                                       ? "more injections than SPH_MAX_INJECT in one update"
                                       : "particle capacity exceeded");
  }
  {
    // maxima of the per-workgroup pairs (non-negative doubles or +inf: their
    // bit patterns order like the values)
    uint64_t b0 = 0, b1 = 0;
    for (int k = 0; k < c->post_blocks; ++k) {
      uint64_t u[2];
      std::memcpy(u, hb + 1040 * 4 + 16 * k, 16);
      b0 = std::max(b0, u[0]);
      b1 = std::max(b1, u[1]);
    }
    std::memcpy(&c->red_v2, &b0, 8);
    std::memcpy(&c->red_nut, &b1, 8);
  }
  int64_t n_inj = cnt[1024], n_del = 0;
  for (int b = 0; b < 256; ++b) n_del += cnt[512 + b];
  c->next_pid = (uint64_t)(uint32_t)cnt[1033] | ((uint64_t)(uint32_t)cnt[1034] << 32);
  c->n_total += n_inj;
  c->n_alive += n_inj - n_del;
  c->n_real += n_inj - n_del;
  c->cells_valid = false;
  c->B_valid = false;
  if (out) {
    std::memcpy(out->n_relabel, cnt, 256 * 4);
    std::memcpy(out->n_inject, cnt + 256, 256 * 4);
    std::memcpy(out->n_delete, cnt + 512, 256 * 4);
    std::memcpy(out->n_revert, cnt + 768, 256 * 4);
    out->n_real = c->n_real;
    out->n_total = c->n_alive;
  }
  sph_status fs = check_flags(c, flags);
  c->red_valid = fs == SPH_OK;
  if (pre) {
    if (fs == SPH_OK) {
      // the prelaunched build and correction hold the updated state (the
      // time-step maxima are over the real particles, which it keeps)
      c->n_total = c->n_alive;
      c->cells_valid = true;
      c->moved = false;
      c->B_valid = true;
    } else {
      // the update's particle arrays stand; the cell arrays were rebuilt
      (void)hipStreamSynchronize(c->stream);
      c->F = saved;
      c->nbr_valid = false;
    }
  }
  return fs;
}

}  // namespace

extern "C" {

size_t sph_workspace_size(const sph_params* params, const sph_buffer_desc* bufs, int32_t nbuf) {
  if (validate(params, bufs, nbuf)) return 0;
  Plan pl;
  make_plan(params, bufs, nbuf, &pl);
  return pl.L.total;
}

sph_status sph_create(const sph_params* params, const sph_buffer_desc* bufs, int32_t nbuf,
                      void* workspace, size_t ws_bytes, void* hip_stream, sph_ctx** out) {
  if (!out) return SPH_E_ARG;
  *out = nullptr;
  const char* msg = validate(params, bufs, nbuf);
  if (msg) return SPH_E_ARG;
  Plan pl;
  make_plan(params, bufs, nbuf, &pl);
  if (!workspace || ws_bytes < pl.L.total || ((uintptr_t)workspace & 255)) return SPH_E_ARG;
  sph_ctx* c = new (std::nothrow) sph_ctx();
  if (!c) return SPH_E_ARG;
  c->P = *params;
  c->nbuf = nbuf;
  c->bufs_h.assign(bufs, bufs + nbuf);
  c->stream = (hipStream_t)hip_stream;
  c->ws = (char*)workspace;
  c->ws_bytes = ws_bytes;
  c->cap = params->capacity;
  (void)hipGetDevice(&c->device);
  // the device address of the library's array for sph_neighbors_noalloc,
  // taken once per device while it is current
  if (noalloc_scratch_init(c->device) != hipSuccess) {
    delete c;
    return SPH_E_HIP;
  }
  grid_of(params, &c->grid);
  if (const char* tl = std::getenv("SPHX_TEAM_LANES")) {   // tuning knob: 1, 2, 4 or 8
    int v = std::atoi(tl);
    if (v == 1 || v == 2 || v == 4 || v == 8) c->team_override = v;
  }
  if (const char* cl = std::getenv("SPHX_CORR_LANES")) {   // tuning knob: 1, 2, 4 or 8
    int v = std::atoi(cl);
    if (v == 1 || v == 2 || v == 4 || v == 8) c->corr_override = v;
  }
  char* w = c->ws;
  Fields& F = c->F;
  for (int k = 0; k < 3; ++k)
    for (int s = 0; s < 2; ++s) {
      F.x[k].a[s] = (double*)(w + pl.off_x[k][s]);
      F.xr[k].a[s] = w + pl.off_xr[k][s];
      F.v[k].a[s] = w + pl.off_v[k][s];
    }
  for (int s = 0; s < 2; ++s) {
    F.rho.a[s] = (double*)(w + pl.off_rho[s]);
    F.drho.a[s] = w + pl.off_drho[s];
    F.k.a[s] = w + pl.off_k[s];
    F.eps.a[s] = w + pl.off_eps[s];
    F.nut.a[s] = w + pl.off_nut[s];
    F.tag.a[s] = (uint32_t*)(w + pl.off_tag[s]);
    F.pid.a[s] = (uint32_t*)(w + pl.off_pid[s]);
    F.p.a[s] = w + pl.off_p[s];
    F.vol.a[s] = w + pl.off_vol[s];
  }
  for (int k = 0; k < 6; ++k) F.B[k] = w + pl.off_B[k];
  for (int k = 0; k < 3; ++k) F.anu[k] = w + pl.off_anu[k];
  F.cell = (int32_t*)(w + pl.off_cell);
  F.nbr = (uint32_t*)(w + pl.off_nbr);
  F.ncnt = (int32_t*)(w + pl.off_ncnt);
  for (int k = 0; k < 3; ++k) F.xrb[k] = w + pl.off_xrb[k];
  for (int k = 0; k < 3; ++k) F.prec[k] = w + pl.off_prec[k];
  for (int k = 0; k < 2; ++k) F.drec[k] = w + pl.off_drec[k];
  for (int k = 0; k < 3; ++k) F.arec[k] = w + pl.off_arec[k];
  for (int k = 0; k < 3; ++k) F.shift[k] = params->tvf_alpha != 0.0 ? w + pl.off_shift[k] : nullptr;
  for (int k = 0; k < 3; ++k) F.cell_u[k] = w + pl.off_cellu[k];
  F.lskin = (float*)(w + pl.off_lskin);
  for (int k = 0; k < 3; ++k)
    F.xr32[k] = (c->P.precision == SPH_FP64 && c->P.dim == 3) ? (float*)(w + pl.off_xr32[k])
                                                                : nullptr;
  F.nbr_k = params->dim == 2 ? kNbrMax2 : kNbrMax3;
  if (const char* nl = std::getenv("SPHX_NBR_LIST")) c->use_nbr = std::atoi(nl) != 0;
  if (const char* tl = std::getenv("SPHX_LIST_TIGHT")) c->tight_list = std::atoi(tl) != 0 ? 1 : 0;
  Scratch& S = c->S;
  S.key = (int32_t*)(w + pl.off_key);
  S.slot = (int32_t*)(w + pl.off_slot);
  S.perm = (int32_t*)(w + pl.off_perm);
  S.dec = (uint32_t*)(w + pl.off_dec);
  S.count = (int32_t*)(w + pl.off_count);
  S.cell_start = (int32_t*)(w + pl.off_cstart);
  S.cell_q = (int32_t*)(w + pl.off_cellq);
  S.block_sums = (int32_t*)(w + pl.off_bsums);
  S.cand_cells = (int32_t*)(w + pl.off_cand);
  S.n_cand_cells = pl.n_cand;
  S.inj_key = (uint64_t*)(w + pl.off_injk);
  S.inj_idx = (int32_t*)(w + pl.off_inji);
  S.counters = (int32_t*)(w + pl.off_counters);
  S.flags = (uint32_t*)(w + pl.off_flags);
  S.stale = (uint32_t*)(w + pl.off_stale);
  S.nstate = (int32_t*)(w + pl.off_nstate);
  S.lrad = (double*)(w + pl.off_lrad);
  S.red = (double*)(w + pl.off_red);
  S.pairs = (long long*)(w + pl.off_pairs);
  S.next_pid = (uint64_t*)(w + pl.off_npid);
  S.bufs = (BufDev*)(w + pl.off_bufs);
  S.bidx = (int32_t*)(w + pl.off_bidx);

  // buffer table with derived values
  c->bufdev_h.resize(kMaxBuf);
  std::vector<int32_t> bidx(256, -1);
  for (int q = 0; q < nbuf; ++q) {
    const sph_buffer_desc& b = bufs[q];
    BufDev& d = c->bufdev_h[q];
    std::memset(&d, 0, sizeof(d));
    d.id = b.id;
    d.vel_mode = b.vel_mode;
    d.p_mode = b.p_mode;
    d.turb_mode = b.turb_mode;
    d.profile = b.profile;
    d.n_coef = b.n_coef;
    for (int k = 0; k < 3; ++k) d.origin[k] = b.origin[k];
    for (int k = 0; k < 9; ++k) d.frame[k] = b.frame[k];
    d.length = b.length;
    d.hw[0] = b.half_width[0];
    d.hw[1] = b.half_width[1];
    d.fringe = b.fringe;
    {
      volatile double L = b.length, f = b.fringe;
      d.gen = L + f;
    }
    d.p_ob = b.p_ob;
    d.k_bc = b.k_bc;
    d.eps_bc = b.eps_bc;
    d.u0 = b.u0;
    d.noise_amp = b.noise_amp;
    d.ramp_time = b.ramp_time;
    {
      volatile double r0 = params->rho0, c0 = params->c0, pob = b.p_ob;
      volatile double den = r0 * c0 * c0;
      volatile double q1 = pob / den;
      volatile double q2 = q1 + 1.0;
      d.rho_bc = r0 * q2;
    }
    for (int m = 0; m < 16; ++m) d.coef[m] = b.coef[m];
    lcll_box(params, c->grid, b, d.clo, d.chi);
    bidx[b.id] = q;
  }
  std::vector<int32_t> cand = candidate_cells(params, c->grid, bufs, nbuf);
  hipStream_t st = c->stream;
  hipError_t e = hipSuccess;
  if (nbuf > 0)
    e = hipMemcpyAsync(S.bufs, c->bufdev_h.data(), sizeof(BufDev) * nbuf, hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(S.bidx, bidx.data(), 256 * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && !cand.empty())
    e = hipMemcpyAsync(S.cand_cells, cand.data(), cand.size() * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemsetAsync(S.flags, 0, 4, st);
  if (e == hipSuccess) e = hipMemsetAsync(S.stale, 0, 8, st);
  if (e == hipSuccess) e = hipMemsetAsync(S.nstate, 0, 16, st);
  if (e == hipSuccess) e = hipMemsetAsync(S.lrad, 0, 32, st);
  if (e == hipSuccess) e = hipMemsetAsync(S.counters, 0, 1040 * 4, st);
  if (e == hipSuccess) e = hipMemsetAsync(S.count, 0, (size_t)c->grid.ncell * 4, st);
  if (e == hipSuccess)
    e = hipMemsetAsync(S.pairs, 0, sizeof(long long) * kPairShards * kPairShardStride, st);
  if (e == hipSuccess) e = hipMemsetAsync(S.next_pid, 0, 8, st);
  // coherent host memory: the post-update reduction writes its read-back
  // here from the device, and the host reads it after the event
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&c->pinned, 1040 * 4 + kPostBlocks * 16, hipHostMallocCoherent);
  if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&c->pinned_dev, c->pinned, 0);
  // a system-scope release when recorded: the device's writes to host
  // memory are visible once the event has completed
  if (e == hipSuccess)
    e = hipEventCreateWithFlags(&c->rb_event, hipEventDisableTiming | hipEventReleaseToSystem);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    if (c->pinned) (void)hipHostFree(c->pinned);
    if (c->rb_event) (void)hipEventDestroy(c->rb_event);
    delete c;
    return SPH_E_HIP;
  }
  *out = c;
  return SPH_OK;
}

sph_status sph_destroy(sph_ctx* c) {
  if (!c) return SPH_E_ARG;
  (void)hipStreamSynchronize(c->stream);
  for (auto& r : c->prof.pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : c->prof.pool) (void)hipEventDestroy(e);
  if (c->pinned) (void)hipHostFree(c->pinned);
  if (c->rb_event) (void)hipEventDestroy(c->rb_event);
  delete c;
  return SPH_OK;
}

const char* sph_last_error(const sph_ctx* c) { return c ? c->err.c_str() : kNoCtx; }

// Tags of n particles read to the host and checked: a buffer particle must
// name a configured buffer (Sec. 3.2).  Nothing is written.
sph_status read_tags(sph_ctx* c, const uint32_t* tag_dev, int64_t n, std::vector<uint32_t>* tags) {
  tags->assign((size_t)n, 0u);
  if (n > 0) {
    HIPCHK(c, hipMemcpyAsync(tags->data(), tag_dev, n * 4, hipMemcpyDeviceToHost, c->stream),
           "tags");
    HIPCHK(c, hipStreamSynchronize(c->stream), "tags sync");
  }
  for (auto t : *tags) {
    if (tag_kind(t) != kBuffer) continue;
    bool known = false;
    for (int q = 0; q < c->nbuf; ++q) known |= c->bufs_h[q].id == (int32_t)tag_bid(t);
    if (!known) return fail(c, SPH_E_ARG, "a buffer particle names an unknown buffer id");
  }
  return SPH_OK;
}

// The state after n particles were written into the live arrays: next id,
// cleared flags, counts, invalid cell list.
sph_status adopt_particles(sph_ctx* c, int64_t n, uint64_t next_pid,
                           const std::vector<uint32_t>& tags) {
  uint64_t np = next_pid;
  HIPCHK(c, hipMemcpyAsync(c->S.next_pid, &np, 8, hipMemcpyHostToDevice, c->stream), "next_pid");
  HIPCHK(c, hipMemsetAsync(c->S.flags, 0, 4, c->stream), "flags");
  HIPCHK(c, hipStreamSynchronize(c->stream), "set_particles sync");
  int64_t real = 0, dead = 0;
  for (auto t : tags) {
    if (tag_kind(t) <= kBuffer) real++;
    if (tag_kind(t) == kDead) dead++;
  }
  c->red_valid = false;
  c->n_total = n;
  c->n_alive = n - dead;
  c->n_real = real;
  c->next_pid = next_pid;
  c->cells_valid = false;
  c->B_valid = false;
  c->moved = false;
  return SPH_OK;
}

sph_status sph_set_particles(sph_ctx* c, int64_t n, uint64_t next_pid, const sph_particles* src) {
  if (!c) return SPH_E_ARG;
  if (!src || n < 0 || n > c->cap) return fail(c, SPH_E_ARG, "bad particle count or source");
  if (n > 0 && (!src->x || !src->v || !src->rho || !src->tag || !src->pid))
    return fail(c, SPH_E_ARG, "x, v, rho, tag and pid are required");
  if (c->P.turbulence && n > 0 && (!src->k || !src->eps))
    return fail(c, SPH_E_ARG, "k and eps are required with turbulence");
  std::vector<uint32_t> tags;
  sph_status st = read_tags(c, src->tag, n, &tags);   // before anything is written
  if (st != SPH_OK) return st;
  HIPCHK(c, launch_set_particles(c, n, src), "set_particles");
  return adopt_particles(c, n, next_pid, tags);
}

sph_status sph_field_offset(const sph_ctx* c, int32_t field, size_t* offset, int32_t* dtype) {
  if (!c || !offset || !dtype) return SPH_E_ARG;
  const Fields& F = c->F;
  const int32_t pt = c->P.precision == SPH_FP64 ? SPH_DTYPE_F64 : SPH_DTYPE_F32;
  const void* p = nullptr;
  int32_t t = SPH_DTYPE_F64;
  switch (field) {
    case SPH_FIELD_X0: case SPH_FIELD_X1: case SPH_FIELD_X2:
      p = F.x[field - SPH_FIELD_X0].live(); break;
    case SPH_FIELD_V0: case SPH_FIELD_V1: case SPH_FIELD_V2:
      p = F.v[field - SPH_FIELD_V0].live(); t = pt; break;
    case SPH_FIELD_RHO: p = F.rho.live(); break;
    case SPH_FIELD_DRHO: p = F.drho.live(); t = pt; break;
    case SPH_FIELD_K: p = F.k.live(); t = pt; break;
    case SPH_FIELD_EPS: p = F.eps.live(); t = pt; break;
    case SPH_FIELD_TAG: p = F.tag.live(); t = SPH_DTYPE_U32; break;
    case SPH_FIELD_PID: p = F.pid.live(); t = SPH_DTYPE_U32; break;
    default: return SPH_E_ARG;
  }
  *offset = (size_t)((const char*)p - c->ws);
  *dtype = t;
  return SPH_OK;
}

sph_status sph_set_count(sph_ctx* c, int64_t n_total, uint64_t next_pid) {
  if (!c) return SPH_E_ARG;
  if (n_total < 0 || n_total > c->cap) return fail(c, SPH_E_ARG, "bad particle count");
  std::vector<uint32_t> tags;
  sph_status st = read_tags(c, c->F.tag.live(), n_total, &tags);
  if (st != SPH_OK) return st;
  HIPCHK(c, launch_derive_nut(c, n_total), "derive nu_t");
  return adopt_particles(c, n_total, next_pid, tags);
}

sph_status sph_get_count(const sph_ctx* c, int64_t* n_total, int64_t* n_real) {
  if (!c) return SPH_E_ARG;
  if (n_total) *n_total = c->n_total;
  if (n_real) *n_real = c->n_real;
  return SPH_OK;
}

sph_status sph_get_particles(sph_ctx* c, const sph_particles* dst) {
  if (!c) return SPH_E_ARG;
  if (!dst) return fail(c, SPH_E_ARG, "dst is NULL");
  HIPCHK(c, launch_get_particles(c, dst), "get_particles");
  HIPCHK(c, hipStreamSynchronize(c->stream), "get_particles sync");
  return SPH_OK;
}

sph_status sph_set_clock(sph_ctx* c, int64_t step, double t) {
  if (!c) return SPH_E_ARG;
  c->step = step;
  c->t = t;
  return SPH_OK;
}

sph_status sph_get_clock(const sph_ctx* c, int64_t* step, double* t, uint64_t* next_pid) {
  if (!c) return SPH_E_ARG;
  if (step) *step = c->step;
  if (t) *t = c->t;
  if (next_pid) *next_pid = c->next_pid;
  return SPH_OK;
}

sph_status sph_build_cells(sph_ctx* c) {
  if (!c) return SPH_E_ARG;
  profile_launch(c, SPH_K_CELLS);
  hipError_t e = launch_build_cells(c, c->n_total, c->n_alive);
  prof_end(c);
  if (e != hipSuccess) return hip_fail(c, e, "build_cells");
  c->n_total = c->n_alive;
  c->cells_valid = true;
  c->moved = false;
  c->B_valid = false;
  c->nbr_valid = false;
  return SPH_OK;
}

sph_status sph_correction(sph_ctx* c) {
  if (!c) return SPH_E_ARG;
  if (!c->cells_valid || c->moved)
    return fail(c, SPH_E_STATE, "sph_correction needs a cell build after the last position change");
  profile_launch(c, SPH_K_CORRECTION);
  // the relative-motion list radius, from the maxima of this state (the
  // last buffer update's when they describe it, else a fresh reduction): the
  // list is the one sph_advance builds for the same state
  const bool tight = list_tight(c);
  hipError_t e = tight ? launch_list_dt(c, !c->red_valid) : hipSuccess;
  if (e == hipSuccess) e = launch_correction(c, nullptr, 0, tight);
  prof_end(c);
  if (e != hipSuccess) return hip_fail(c, e, "correction");
  c->B_valid = true;
  return SPH_OK;
}

sph_status sph_step(sph_ctx* c, const sph_step_ctrl* ctrl, sph_step_info* out) {
  if (!c) return SPH_E_ARG;
  if (!c->cells_valid || c->moved || !c->B_valid)
    return fail(c, SPH_E_STATE, "sph_step needs sph_build_cells and sph_correction first");
  if (ctrl && ctrl->dt_adv > 0 && ctrl->n_ac < 1) return fail(c, SPH_E_ARG, "ctrl->n_ac must be >= 1");
  double v2max, nutmax;
  hipError_t e;
  if (c->red_valid) {
    // reduced, and flags checked, by the buffer update that produced this state
    v2max = c->red_v2;
    nutmax = c->red_nut;
  } else {
    double* host = (double*)c->pinned;
    profile_launch(c, SPH_K_REDUCE);
    e = launch_reduce(c, host);
    prof_end(c);
    if (e != hipSuccess) return hip_fail(c, e, "reduce");
    HIPCHK(c, hipStreamSynchronize(c->stream), "step sync");
    if (c->prof.on) resolve_events(c);
    uint32_t flags = *(uint32_t*)(host + 2);
    sph_status fs = check_flags(c, flags);
    if (fs != SPH_OK) return fs;
    v2max = host[0];
    nutmax = host[1];
  }
  c->red_valid = false;
  if (!std::isfinite(v2max) || !std::isfinite(nutmax))
    return fail(c, SPH_E_NUMERIC, "non-finite velocity or density");
  const sph_params& P = c->P;
  // dual-criteria time step (Sec. 2.3; criteria are a reading of the cited scheme)
  const double vmax = std::sqrt(v2max);
  const double numax = P.nu_l + nutmax;
  const double h = P.h;
  double dt_adv = P.cfl_adv * std::fmin(h / std::fmax(vmax, P.u_ref), h * h / (2.0 * numax));
  const double dt_ac = P.cfl_ac * h / (P.c0 + vmax);
  int n_ac = (int)std::ceil(dt_adv / dt_ac);
  if (n_ac < 1) n_ac = 1;
  if (ctrl && ctrl->dt_adv > 0) {
    dt_adv = ctrl->dt_adv;
    n_ac = ctrl->n_ac;
  }
  const double dt = dt_adv / n_ac;

  profile_launch(c, SPH_K_ADVECTION);
  e = launch_advection(c, dt_adv, dt, false, nullptr);
  prof_end(c);
  if (e != hipSuccess) return hip_fail(c, e, "advection");
  c->F.p.flip();
  c->F.vol.flip();
  if (P.turbulence) {
    c->F.k.flip();
    c->F.eps.flip();
    c->F.nut.flip();
  }
  for (int s = 0; s < n_ac; ++s) {
    c->substep = s;
    profile_launch(c, SPH_K_PRESSURE);
    e = launch_pressure(c, dt, false, nullptr);
    prof_end(c);
    if (e != hipSuccess) return hip_fail(c, e, "pressure");
    profile_launch(c, SPH_K_DENSITY);
    e = launch_density(c, dt, s == n_ac - 1, false, nullptr);
    prof_end(c);
    if (e != hipSuccess) return hip_fail(c, e, "density");
  }
  if (c->F.shift[0]) {   // transport-velocity shift of the start-of-step state
    e = launch_shift_apply(c);
    if (e != hipSuccess) return hip_fail(c, e, "shift");
  }
  c->step += 1;
  c->t += dt_adv;
  c->moved = true;
  c->B_valid = false;
  if (out) {
    out->dt_adv = dt_adv;
    out->dt_ac = dt;
    out->vmax = vmax;
    out->numax = numax;
    out->t = c->t;
    out->n_ac = n_ac;
    out->list_outgrown = -1;   // known after the next buffer update (sph_advance)
    out->step = c->step;
  }
  return SPH_OK;
}

sph_status sph_advance(sph_ctx* c, const sph_step_ctrl* ctrl, sph_step_info* info,
                       sph_buffer_counts* counts) {
  if (!c) return SPH_E_ARG;
  sph_status st = SPH_OK;
  // a state left by the previous sph_advance is already built and corrected
  // (building a built state again is the identity)
  if (!(c->cells_valid && c->B_valid && !c->moved)) {
    st = sph_build_cells(c);
    if (st == SPH_OK) st = sph_correction(c);
  }
  if (st == SPH_OK) st = sph_step(c, ctrl, info);
  if (st == SPH_OK) st = buffer_update(c, nullptr, nullptr, 0, counts, true);
  if (st == SPH_OK && info) info->list_outgrown = c->last_outgrown ? 1 : 0;
  return st;
}

sph_status sph_buffer_update(sph_ctx* c, sph_buffer_counts* out) {
  return buffer_update(c, nullptr, nullptr, 0, out, false);
}

sph_status sph_buffer_update_ex(sph_ctx* c, const uint32_t* forced_by_pid, uint32_t* log_by_pid,
                                int64_t pid_cap, sph_buffer_counts* out) {
  return buffer_update(c, forced_by_pid, log_by_pid, pid_cap, out, false);
}

sph_status sph_buffer_decisions(sph_ctx* c, uint32_t* dec) {
  if (!c) return SPH_E_ARG;
  if (!dec) return fail(c, SPH_E_ARG, "dec is NULL");
  if (!c->cells_valid) return fail(c, SPH_E_STATE, "sph_buffer_decisions needs sph_build_cells");
  HIPCHK(c, launch_zero_i32(c, (int32_t*)dec, c->n_total), "zero");
  HIPCHK(c, launch_buffer_decide(c, true, dec), "decide");
  HIPCHK(c, hipStreamSynchronize(c->stream), "decide sync");
  return SPH_OK;
}

sph_status sph_eval_rates(sph_ctx* c, const sph_rates* out) {
  if (!c) return SPH_E_ARG;
  if (!out) return fail(c, SPH_E_ARG, "out is NULL");
  if (!c->cells_valid || c->moved || !c->B_valid)
    return fail(c, SPH_E_STATE, "sph_eval_rates needs sph_build_cells and sph_correction");
  if (c->B_pending) HIPCHK(c, launch_moment(c), "moment");   // a state left by sph_advance
  HIPCHK(c, launch_prepare_pv(c, out), "prepare_pv");
  if (out->anu || out->gradv || out->dk || out->deps || out->shift)
    HIPCHK(c, launch_advection(c, 0.0, 0.0, true, out), "advection rates");
  if (out->ap) HIPCHK(c, launch_pressure(c, 0.0, true, out), "pressure rates");
  if (out->drho) HIPCHK(c, launch_density(c, 0.0, false, true, out), "density rates");
  if (out->B) HIPCHK(c, launch_export_B(c, out->B), "export B");
  return SPH_OK;
}

sph_status sph_neighbors(sph_ctx* c, int32_t* row_ptr, int32_t* col, int64_t cap, int64_t* n_pairs) {
  if (!c) return SPH_E_ARG;
  if (!row_ptr || !n_pairs || cap < 0 || (cap > 0 && !col))
    return fail(c, SPH_E_ARG, "bad neighbour arguments");
  if (!c->cells_valid || c->moved)
    return fail(c, SPH_E_STATE, "sph_neighbors needs a cell build after the last position change");
  HIPCHK(c, launch_neighbors(c, row_ptr, col, cap, n_pairs), "neighbors");
  HIPCHK(c, hipStreamSynchronize(c->stream), "neighbors sync");
  if (*n_pairs > cap) return fail(c, SPH_E_CAPACITY, "neighbour list longer than cap");
  return SPH_OK;
}

sph_status sph_neighbors_noalloc(sph_ctx* c, int32_t* row_ptr, int32_t* col, int64_t cap,
                                 int64_t* n_pairs) {
  if (!c) return SPH_E_ARG;
  if (!row_ptr || !n_pairs || cap < 0 || (cap > 0 && !col))
    return fail(c, SPH_E_ARG, "bad neighbour arguments");
  if (c->n_total > SPH_NOALLOC_MAX_PARTICLES)
    return fail(c, SPH_E_ARG, "more particles than SPH_NOALLOC_MAX_PARTICLES");
  if (!c->cells_valid || c->moved)
    return fail(c, SPH_E_STATE, "sph_neighbors_noalloc needs a cell build after the last position change");
  HIPCHK(c, launch_neighbors_noalloc(c, row_ptr, col, cap, n_pairs), "neighbors_noalloc");
  HIPCHK(c, hipStreamSynchronize(c->stream), "neighbors_noalloc sync");
  if (*n_pairs > cap) return fail(c, SPH_E_CAPACITY, "neighbour list longer than cap");
  return SPH_OK;
}

sph_status sph_step_pairs(sph_ctx* c, int32_t* row_ptr, int32_t* col, int64_t cap,
                          int64_t* n_pairs) {
  if (!c) return SPH_E_ARG;
  if (!row_ptr || !n_pairs || cap < 0 || (cap > 0 && !col))
    return fail(c, SPH_E_ARG, "bad pair-list arguments");
  if (!c->cells_valid || c->moved || !c->B_valid)
    return fail(c, SPH_E_STATE, "sph_step_pairs needs sph_build_cells and sph_correction");
  HIPCHK(c, launch_walk_pairs(c, row_ptr, col, cap, n_pairs), "step pairs");
  HIPCHK(c, hipStreamSynchronize(c->stream), "step pairs sync");
  if (*n_pairs > cap) return fail(c, SPH_E_CAPACITY, "pair list longer than cap");
  return SPH_OK;
}

sph_status sph_profile_enable(sph_ctx* c, int32_t on) {
  if (!c) return SPH_E_ARG;
  c->prof.on = on != 0;
  return SPH_OK;
}

sph_status sph_profile_read(sph_ctx* c, int32_t kernel, sph_kernel_stats* out) {
  if (!c) return SPH_E_ARG;
  if (kernel < 0 || kernel >= SPH_K_COUNT || !out) return fail(c, SPH_E_ARG, "bad kernel id");
  HIPCHK(c, hipStreamSynchronize(c->stream), "profile sync");
  resolve_events(c);
  out->total_ms = c->prof.total_ms[kernel];
  out->launches = c->prof.launches[kernel];
  out->bytes = c->prof.bytes[kernel];
  out->particles = c->prof.particles[kernel];
  return SPH_OK;
}

sph_status sph_pair_count(sph_ctx* c, int64_t* pairs) {
  if (!c || !pairs) return SPH_E_ARG;
  const size_t bytes = sizeof(long long) * kPairShards * kPairShardStride;
  std::vector<long long> v((size_t)kPairShards * kPairShardStride);
  HIPCHK(c, hipMemcpyAsync(v.data(), c->S.pairs, bytes, hipMemcpyDeviceToHost, c->stream), "pairs");
  HIPCHK(c, hipMemsetAsync(c->S.pairs, 0, bytes, c->stream), "pairs reset");
  HIPCHK(c, hipStreamSynchronize(c->stream), "pairs sync");
  long long s = 0;
  for (int k = 0; k < kPairShards; ++k) s += v[(size_t)k * kPairShardStride];
  *pairs = s;
  return SPH_OK;
}

sph_status sph_set_profile_coef(sph_ctx* c, int32_t buffer_id, int32_t n_coef, const double* coef) {
  if (!c) return SPH_E_ARG;
  if (n_coef < 0 || n_coef > 16 || (n_coef > 0 && !coef))
    return fail(c, SPH_E_ARG, "n_coef must be 0..16 with a coefficient array");
  int q = -1;
  for (int k = 0; k < c->nbuf; ++k)
    if (c->bufs_h[k].id == buffer_id) q = k;
  if (q < 0) return fail(c, SPH_E_ARG, "no buffer with this id");
  BufDev& d = c->bufdev_h[q];
  d.n_coef = n_coef;
  c->bufs_h[q].n_coef = n_coef;
  for (int m = 0; m < 16; ++m) {
    d.coef[m] = m < n_coef ? coef[m] : 0.0;
    c->bufs_h[q].coef[m] = d.coef[m];
  }
  HIPCHK(c, hipMemcpyAsync(c->S.bufs + q, &d, sizeof(BufDev), hipMemcpyHostToDevice, c->stream),
         "profile coefficients");
  HIPCHK(c, hipStreamSynchronize(c->stream), "profile sync");
  return SPH_OK;
}

sph_status sph_objective(sph_ctx* c, const sph_objective_desc* obj, const uint8_t* member_by_pid,
                         uint8_t* member_out_by_pid, int64_t pid_cap, double* J) {
  if (!c) return SPH_E_ARG;
  if (!obj || !J) return fail(c, SPH_E_ARG, "obj and J are required");
  if (c->P.turbulence) return fail(c, SPH_E_ARG, "the objectives are defined for laminar runs");
  if (!(obj->slab_width > 0) || !(obj->wall_length > 0))
    return fail(c, SPH_E_ARG, "slab_width and wall_length must be > 0");
  if ((member_by_pid || member_out_by_pid) && pid_cap < (int64_t)c->next_pid)
    return fail(c, SPH_E_ARG, "pid_cap must cover every particle id (>= next_pid)");
  if (!c->cells_valid) return fail(c, SPH_E_STATE, "sph_objective needs the cell list of the step");
  HIPCHK(c, launch_objective(c, obj, member_by_pid, member_out_by_pid, pid_cap, J), "objective");
  return SPH_OK;
}

size_t sph_adjoint_workspace_size(const sph_ctx* c, int32_t max_nac) {
  if (!c) return 0;
  return adjoint_ws_bytes(c, max_nac);
}

}  // extern "C"

namespace {

sph_status adjoint_check(sph_ctx* c, const sph_adjoint_ctrl* ctl, const void* adj_ws,
                         size_t adj_bytes) {
  if (!ctl) return fail(c, SPH_E_ARG, "null argument");
  if (c->P.turbulence) return fail(c, SPH_E_ARG, "the adjoint needs a laminar context");
  if (c->P.tvf_alpha != 0.0)
    return fail(c, SPH_E_ARG, "the adjoint is defined without the transport-velocity shift");
  if (ctl->n_ac < 1 || !(ctl->dt_adv > 0)) return fail(c, SPH_E_ARG, "bad dt_adv / n_ac");
  if (!ctl->dec_by_pid || ctl->pid_cap < (int64_t)ctl->next_pid)
    return fail(c, SPH_E_ARG, "dec_by_pid with pid_cap >= next_pid is required");
  const size_t need = adjoint_ws_bytes(c, ctl->n_ac);
  if (!adj_ws || adj_bytes < need || ((uintptr_t)adj_ws & 255))
    return fail(c, SPH_E_ARG, "adjoint workspace too small or not 256-byte aligned");
  return SPH_OK;
}

// The recorded step from the context's state, keeping its sub-step states
// and its build, list, correction and update data in the workspace.
sph_status adjoint_forward(sph_ctx* c, const sph_adjoint_ctrl* ctl, char* ws, int64_t* n_step) {
  const int N = ctl->n_ac;
  const double dt = ctl->dt_adv / N;
  c->step = ctl->step;
  c->t = ctl->t;
  sph_status st = sph_build_cells(c);
  if (st != SPH_OK) return st;
  if ((st = sph_correction(c)) != SPH_OK) return st;
  HIPCHK(c, adjoint_snap_start(c, ws, N), "adjoint snapshot");
  HIPCHK(c, launch_advection(c, ctl->dt_adv, dt, false, nullptr), "advection");
  c->F.p.flip();
  c->F.vol.flip();
  HIPCHK(c, adjoint_snap_advection(c, ws, N), "adjoint snapshot");
  for (int s = 0; s < N; ++s) {
    c->substep = s;
    HIPCHK(c, launch_pressure(c, dt, false, nullptr), "pressure");
    HIPCHK(c, adjoint_snap_pressure(c, ws, N, s), "adjoint snapshot");
    HIPCHK(c, launch_density(c, dt, s == N - 1, false, nullptr), "density");
    HIPCHK(c, adjoint_snap_density(c, ws, N, s), "adjoint snapshot");
  }
  c->step += 1;
  c->t += ctl->dt_adv;
  c->moved = true;
  c->B_valid = false;
  const int n = (int)c->n_total;
  if ((st = sph_buffer_update_ex(c, ctl->dec_by_pid, nullptr, ctl->pid_cap, nullptr)) != SPH_OK)
    return st;
  HIPCHK(c, adjoint_keep_step(c, ws, N, n), "adjoint snapshot");
  *n_step = n;
  return SPH_OK;
}

sph_status adjoint_reverse(sph_ctx* c, const sph_objective_desc* obj, const sph_adjoint_ctrl* ctl,
                           int64_t n_step, double* lam, double* grad, char* ws) {
  HIPCHK(c, adjoint_reverse_launch(c, ws, obj, ctl, (int)n_step, lam, grad), "adjoint");
  HIPCHK(c, hipMemcpyAsync((char*)c->pinned + 64, c->S.flags, 4, hipMemcpyDeviceToHost, c->stream),
         "flags");
  HIPCHK(c, hipStreamSynchronize(c->stream), "adjoint sync");
  const uint32_t flags = *(uint32_t*)((char*)c->pinned + 64);
  if (flags & kFlagCapacity) return fail(c, SPH_E_ARG, "a particle id is not below pid_cap");
  return check_flags(c, flags);
}

}  // namespace

extern "C" {

sph_status sph_adjoint_forward(sph_ctx* c, const sph_adjoint_ctrl* ctl, void* adj_ws,
                               size_t adj_bytes, int64_t* n_step) {
  if (!c) return SPH_E_ARG;
  if (!n_step) return fail(c, SPH_E_ARG, "null argument");
  sph_status st = adjoint_check(c, ctl, adj_ws, adj_bytes);
  if (st != SPH_OK) return st;
  if (c->next_pid != ctl->next_pid)
    return fail(c, SPH_E_STATE, "the context is not at the recorded step's start (next_pid)");
  return adjoint_forward(c, ctl, (char*)adj_ws, n_step);
}

sph_status sph_adjoint_reverse(sph_ctx* c, const sph_objective_desc* obj,
                               const sph_adjoint_ctrl* ctl, int64_t n_step, double* lam,
                               double* grad, void* adj_ws, size_t adj_bytes) {
  if (!c) return SPH_E_ARG;
  if (!obj || !lam || !grad) return fail(c, SPH_E_ARG, "null argument");
  sph_status st = adjoint_check(c, ctl, adj_ws, adj_bytes);
  if (st != SPH_OK) return st;
  if (n_step < 0 || n_step > c->cap) return fail(c, SPH_E_ARG, "bad n_step");
  if (!(obj->slab_width > 0) || !(obj->wall_length > 0))
    return fail(c, SPH_E_ARG, "slab_width and wall_length must be > 0");
  return adjoint_reverse(c, obj, ctl, n_step, lam, grad, (char*)adj_ws);
}

sph_status sph_adjoint_step(sph_ctx* c, const sph_particles* pre, int64_t n_pre,
                            const sph_objective_desc* obj, const sph_adjoint_ctrl* ctl,
                            double* lam, double* grad, void* adj_ws, size_t adj_bytes) {
  if (!c) return SPH_E_ARG;
  if (!pre || !obj || !ctl || !lam || !grad) return fail(c, SPH_E_ARG, "null argument");
  sph_status st = adjoint_check(c, ctl, adj_ws, adj_bytes);
  if (st != SPH_OK) return st;
  if (!(obj->slab_width > 0) || !(obj->wall_length > 0))
    return fail(c, SPH_E_ARG, "slab_width and wall_length must be > 0");
  // replay the step from its start state, then walk it backwards
  if ((st = sph_set_particles(c, n_pre, ctl->next_pid, pre)) != SPH_OK) return st;
  int64_t n_step = 0;
  if ((st = adjoint_forward(c, ctl, (char*)adj_ws, &n_step)) != SPH_OK) return st;
  return adjoint_reverse(c, obj, ctl, n_step, lam, grad, (char*)adj_ws);
}

}  // extern "C"
