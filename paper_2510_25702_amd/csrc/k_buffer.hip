// Bidirectional buffer update on gfx950 (Secs. 2.4.2, 2.4.3, 3.1, 3.2 of the
// paper).  Only particles in the candidate cells (each buffer's local
// cell-linked-list box, widened by one cell for the drift since the cell
// build) are examined, one wavefront per cell:
//   K12 decide: every decision from one snapshot, FP64 predicates without
//       contraction (a decision reads only its own particle, so its tag
//       change -- relabel, revert, dead for a deletion, which the next cell
//       build drops: the counting sort is the compaction -- is applied at
//       once); injections are appended to a short list (integer atomic on a
//       counter, order fixed afterwards by sorting);
//   K13 inject (one workgroup): bitonic sort of the list by (buffer id,
//       parent id), in the registers of one wavefront for up to 64 entries
//       and in LDS beyond, capacity check, append the new fluid particles at
//       the end of the arrays, recycle the parents by -L_b n_b (Eq.
//       (eq-pos-new-added)) with the buffer's boundary values;
//   undo: when the injections do not fit, the tag changes are reverted from
//       the recorded decision codes and the update fails as a whole.
#include "sph_ctx.h"

namespace sphx {

namespace {

template <typename T>
T* tp(void* p) { return static_cast<T*>(p); }

struct BufArgs {
  const double* x[3];
  uint32_t* tag;
  const uint32_t* pid;
  uint32_t* dec;
  const BufDev* bufs;
  const int32_t* bidx;
  const int32_t* cand;
  const int32_t* cstart;
  int nbuf, dim;
  GridDev g;
  int32_t* counters;  // relabel[256] inject[256] delete[256] revert[256] n_inj
  uint64_t* inj_key;
  int32_t* inj_idx;
  uint32_t* flags;
  int dry;
  uint32_t* dec_out;
  const uint32_t* forced;   // decisions by particle id (replay), or NULL
  uint32_t* log;            // decisions by particle id (record), or NULL
  int64_t pid_cap;          // length of forced / log
  int n;                    // particle slots (forced replay: every slot)
  double two_h;             // kernel support 2h
};

__device__ __forceinline__ bool in_box(const int c[3], const BufDev& b, int dim) {
  for (int k = 0; k < dim; ++k)
    if (c[k] < b.clo[k] || c[k] > b.chi[k]) return false;
  return true;
}

__device__ __forceinline__ bool in_region(int dim, const BufDev& b, const double y[3]) {
  return y[0] >= 0.0 && y[0] <= b.length && contained(dim, b, y);
}

__device__ uint32_t decide(const BufArgs& a, double x0, double x1, double x2, uint32_t tag) {
  const uint32_t kind = tag_kind(tag);
  if (kind != kFluid && kind != kBuffer) return kDecNone;
  const double xs[3] = {x0, x1, x2};
  int c[3] = {0, 0, 0};
  for (int k = 0; k < a.dim; ++k) c[k] = cell_coord(xs[k], a.g.lo[k], a.g.cs);
  double y[3];
  if (kind == kBuffer) {
    const int q = a.bidx[tag_bid(tag)];
    if (q < 0) return kDecNone;
    const BufDev& b = a.bufs[q];
    if (!in_box(c, b, a.dim)) return kDecNone;
    to_local(b, x0, x1, x2, y);
    if (contained(a.dim, b, y)) {
      if (y[0] < 0.0) return kDecDelete | ((uint32_t)b.id << 8);
      if (y[0] >= b.gen) return kDecInject | ((uint32_t)b.id << 8);
      return kDecNone;
    }
    for (int q2 = 0; q2 < a.nbuf; ++q2) {
      const BufDev& b2 = a.bufs[q2];
      if (!in_box(c, b2, a.dim)) continue;
      double y2[3];
      to_local(b2, x0, x1, x2, y2);
      if (in_region(a.dim, b2, y2))
        return kDecRevertRelabel | ((uint32_t)b.id << 8) | ((uint32_t)b2.id << 16);
    }
    // out through a side of its box into no region and behind the open-face
    // plane of a buffer whose face, extended along its plane by this
    // particle's buffer length to the generation line and by 2h, reaches it:
    // it left the domain at a corner of two open boundaries.  A far plane
    // (a channel bent by more than 180 degrees) does not delete it.
    const double m = __dadd_rn(b.gen, a.two_h);
    for (int q2 = 0; q2 < a.nbuf; ++q2) {
      const BufDev& b2 = a.bufs[q2];
      double y2[3];
      to_local(b2, x0, x1, x2, y2);
      if (!(y2[0] < 0.0)) continue;
      if (fabs(y2[1]) > __dadd_rn(b2.hw[0], m)) continue;
      if (a.dim == 3 && fabs(y2[2]) > __dadd_rn(b2.hw[1], m)) continue;
      return kDecDelete | ((uint32_t)b.id << 8);
    }
    return kDecRevert | ((uint32_t)b.id << 8);
  }
  for (int q = 0; q < a.nbuf; ++q) {
    const BufDev& b = a.bufs[q];
    if (!in_box(c, b, a.dim)) continue;
    to_local(b, x0, x1, x2, y);
    if (in_region(a.dim, b, y)) return kDecRelabel | ((uint32_t)b.id << 8);
  }
  return kDecNone;
}

// Tag change of a decision, applied by the decide kernels with the decision
// (undone by undo_one when the injections fail).
__device__ __forceinline__ void apply_one(const BufArgs& a, int i, uint32_t d) {
  const uint32_t act = d & 0xFFu, id = (d >> 8) & 0xFFu, id2 = (d >> 16) & 0xFFu;
  if (act == kDecRelabel) a.tag[i] = kBuffer | (id << 8);
  else if (act == kDecRevert) a.tag[i] = kFluid;
  else if (act == kDecRevertRelabel) a.tag[i] = kBuffer | (id2 << 8);
  else if (act == kDecDelete) a.tag[i] = kDead;
}

// Count a decision and queue an injection.
__device__ __forceinline__ void record(const BufArgs& a, int i, uint32_t d) {
  a.dec[i] = d;
  const uint32_t act = d & 0xFFu, id = (d >> 8) & 0xFFu, id2 = (d >> 16) & 0xFFu;
  switch (act) {
    case kDecRelabel: atomicAdd(&a.counters[id], 1); break;
    case kDecInject: {
      atomicAdd(&a.counters[256 + id], 1);
      const int slot = atomicAdd(&a.counters[1024], 1);
      if (slot < kMaxInject) {
        a.inj_key[slot] = ((uint64_t)id << 32) | (uint64_t)a.pid[i];
        a.inj_idx[slot] = i;
      }
      break;
    }
    case kDecDelete: atomicAdd(&a.counters[512 + id], 1); break;
    case kDecRevert: atomicAdd(&a.counters[768 + id], 1); break;
    case kDecRevertRelabel:
      atomicAdd(&a.counters[768 + id], 1);
      atomicAdd(&a.counters[id2], 1);
      break;
    default: break;
  }
}

// K12: one wavefront per candidate cell.
__global__ __launch_bounds__(kWave) void k_buffer_decide(BufArgs a) {
  const int cell = a.cand[blockIdx.x];
  const int b = a.cstart[cell], e = a.cstart[cell + 1];
  for (int i = b + (int)threadIdx.x; i < e; i += kWave) {
    const uint32_t d = decide(a, a.x[0][i], a.x[1][i], a.x[2][i], a.tag[i]);
    if (a.dry) {
      a.dec_out[i] = d;
      continue;
    }
    if (a.log && a.pid[i] < a.pid_cap) a.log[a.pid[i]] = d;
    record(a, i, d);
    apply_one(a, i, d);   // a decision reads only its own particle's tag
  }
}

// K12 (replay): the decisions of a recorded update, looked up by particle id
// for every slot, in place of the predicates.
__global__ __launch_bounds__(256) void k_buffer_forced(BufArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const uint32_t p = a.pid[i];
  uint32_t d = p < a.pid_cap ? a.forced[p] : kDecNone;
  if (!is_real(a.tag[i])) d = kDecNone;
  if (a.log && p < a.pid_cap) a.log[p] = d;
  record(a, i, d);
  apply_one(a, i, d);
}

// The decide kernels apply the tag changes at once; when the injection
// then fails for capacity they are undone (every code records the tag it
// replaced: relabel from FLUID, revert / delete from BUFFER(b)).
__device__ __forceinline__ void undo_one(const BufArgs& a, int i) {
  const uint32_t d = a.dec[i];
  const uint32_t act = d & 0xFFu, id = (d >> 8) & 0xFFu;
  if (act == kDecRelabel) a.tag[i] = kFluid;
  else if (act == kDecRevert || act == kDecRevertRelabel || act == kDecDelete)
    a.tag[i] = kBuffer | (id << 8);
}

__global__ __launch_bounds__(kWave) void k_buffer_undo(BufArgs a) {
  const int cell = a.cand[blockIdx.x];
  const int b = a.cstart[cell], e = a.cstart[cell + 1];
  for (int i = b + (int)threadIdx.x; i < e; i += kWave) undo_one(a, i);
}

__global__ __launch_bounds__(256) void k_buffer_undo_all(BufArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < a.n) undo_one(a, i);
}

template <typename T>
struct InjArgs {
  double* x[3];
  T* v[3];
  double* rho;
  T* drho;
  T *k, *eps, *nut;
  uint32_t* tag;
  uint32_t* pid;
  const BufDev* bufs;
  const int32_t* bidx;
  int32_t* counters;
  uint64_t* inj_key;
  int32_t* inj_idx;
  uint64_t* next_pid;
  uint32_t* flags;
  int64_t n, cap;
  int dim, turb;
  double Cmu, rho0, c0;
  uint64_t seed;
  int64_t step;
  double t;
};

constexpr int kInjThreads = 1024;
static_assert(kInjThreads <= kMaxInject, "the first keys are loaded one per thread");

// Child r of the update (rank r in the sorted list) of parent i: an exact
// copy of i appended at slot n + r with particle id base_pid + r; the parent
// is then recycled by -L_b n_b with the buffer's boundary values.  One
// thread per child, so each parent's fields are read once.
template <typename T>
__device__ __forceinline__ void inject_one(const InjArgs<T>& a, const BufDev& b, int r, int i,
                                           uint64_t base_pid) {
  const int64_t c = a.n + r;
  double x[3];
  T v[3];
  for (int k = 0; k < 3; ++k) {
    x[k] = a.x[k][i];
    v[k] = a.v[k][i];
  }
  const double rho = a.rho[i];
  const T drho = a.drho[i];
  const uint32_t pid = a.pid[i];
  T kt = T(0), et = T(0), nt = T(0);
  if (a.turb) {
    kt = a.k[i];
    et = a.eps[i];
    nt = a.nut[i];
  }
  for (int k = 0; k < 3; ++k) {
    a.x[k][c] = x[k];
    a.v[k][c] = v[k];
  }
  a.rho[c] = rho;
  a.drho[c] = drho;
  if (a.turb) {
    a.k[c] = kt;
    a.eps[c] = et;
    a.nut[c] = nt;
  }
  a.tag[c] = kFluid;
  a.pid[c] = (uint32_t)(base_pid + (uint64_t)r);
  double xn[3];
  for (int k = 0; k < 3; ++k) {
    const double tt = __dmul_rn(b.length, b.frame[k]);
    xn[k] = __dsub_rn(x[k], tt);
    a.x[k][i] = xn[k];
  }
  if (b.vel_mode == kVelPrescribed) {
    double y[3];
    to_local(b, xn[0], xn[1], xn[2], y);
    const double u = profile_speed(a.dim, b, y, a.seed, pid, a.step, a.t);
    for (int k = 0; k < 3; ++k) a.v[k][i] = (T)(u * b.frame[k]);
  }
  if (b.p_mode == kPPrescribed)
    a.rho[i] = rho_of_p(a.rho0, a.c0, __dmul_rn(b.p_ob, buffer_ramp(b, a.t)));
  if (a.turb && b.turb_mode == kTurbFreestream) {
    a.k[i] = (T)b.k_bc;
    a.eps[i] = (T)b.eps_bc;
    a.nut[i] = (T)(a.Cmu * b.k_bc * b.k_bc / b.eps_bc);
  }
}

// K13: one workgroup.  The count, the first keys, the next particle id and
// the buffer index table are loaded together; up to one wavefront of
// injections (the usual case) is sorted in registers by that wavefront,
// more in LDS by the whole workgroup.  The sorted order is kept in inj_idx:
// child r of this update is the copy of slot inj_idx[r].
template <typename T>
__global__ __launch_bounds__(kInjThreads) void k_buffer_inject(InjArgs<T> a) {
  __shared__ uint64_t skey[kMaxInject];
  __shared__ int32_t sidx[kMaxInject];
  __shared__ int32_t sbidx[256];
  const int t = threadIdx.x;
  const int m = a.counters[1024];
  const uint64_t base_pid = *a.next_pid;
  const uint64_t key0 = a.inj_key[t];
  const int32_t idx0 = a.inj_idx[t];
  if (t < 256) sbidx[t] = a.bidx[t];
  if (m > kMaxInject || a.n + m > a.cap) {
    if (t == 0) atomicOr(a.flags, kFlagCapacity | (m > kMaxInject ? kFlagInjectOverflow : 0u));
    return;
  }
  if (m == 0) return;
  __syncthreads();
  if (m <= kWave) {
    if (t >= kWave) return;
    // bitonic network over the 64 lanes, padded with the largest key
    uint64_t key = t < m ? key0 : ~0ull;
    int idx = t < m ? idx0 : -1;
#pragma unroll
    for (int kk = 2; kk <= kWave; kk <<= 1) {
#pragma unroll
      for (int jj = kk >> 1; jj > 0; jj >>= 1) {
        const uint64_t ok = lane_xor_by(key, jj);
        const int oi = lane_xor_by(idx, jj);
        const bool up = (t & kk) == 0, low = (t & jj) == 0;
        if (low == up ? ok < key : ok > key) {
          key = ok;
          idx = oi;
        }
      }
    }
    if (t < m) {
      a.inj_idx[t] = idx;
      inject_one(a, a.bufs[sbidx[(int)(key >> 32)]], t, idx, base_pid);
    }
    if (t == 0) *a.next_pid = base_pid + (uint64_t)m;
    return;
  }
  int np2 = 1;
  while (np2 < m) np2 <<= 1;
  for (int r = t; r < np2; r += kInjThreads) {
    const bool own = r == t;
    skey[r] = r < m ? (own ? key0 : a.inj_key[r]) : ~0ull;
    sidx[r] = r < m ? (own ? idx0 : a.inj_idx[r]) : -1;
  }
  __syncthreads();
  for (int kk = 2; kk <= np2; kk <<= 1) {
    for (int jj = kk >> 1; jj > 0; jj >>= 1) {
      for (int r = t; r < np2; r += kInjThreads) {
        const int p = r ^ jj;
        if (p > r) {
          const bool up = (r & kk) == 0;
          const uint64_t kr = skey[r], kp = skey[p];
          if ((kr > kp) == up) {
            skey[r] = kp;
            skey[p] = kr;
            const int s = sidx[r];
            sidx[r] = sidx[p];
            sidx[p] = s;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int r = t; r < m; r += kInjThreads) {
    const int i = sidx[r];
    a.inj_idx[r] = i;
    inject_one(a, a.bufs[sbidx[(int)(skey[r] >> 32)]], r, i, base_pid);
  }
  if (t == 0) *a.next_pid = base_pid + (uint64_t)m;
}

BufArgs make_bufargs(sph_ctx* c, bool dry, uint32_t* dec_out) {
  BufArgs a;
  for (int k = 0; k < 3; ++k) a.x[k] = c->F.x[k].live();
  a.tag = c->F.tag.live();
  a.pid = c->F.pid.live();
  a.dec = c->S.dec;
  a.bufs = c->S.bufs;
  a.bidx = c->S.bidx;
  a.cand = c->S.cand_cells;
  a.cstart = c->S.cell_start;
  a.nbuf = c->nbuf;
  a.dim = c->P.dim;
  a.g = c->grid;
  a.counters = c->S.counters;
  a.inj_key = c->S.inj_key;
  a.inj_idx = c->S.inj_idx;
  a.flags = c->S.flags;
  a.dry = dry ? 1 : 0;
  a.dec_out = dec_out;
  a.forced = nullptr;
  a.log = nullptr;
  a.pid_cap = 0;
  a.n = (int)c->n_total;
  a.two_h = 2.0 * c->P.h;
  return a;
}

template <typename T>
hipError_t inject_impl(sph_ctx* c) {
  InjArgs<T> a;
  Fields& F = c->F;
  for (int k = 0; k < 3; ++k) {
    a.x[k] = F.x[k].live();
    a.v[k] = tp<T>(F.v[k].live());
  }
  a.rho = F.rho.live();
  a.drho = tp<T>(F.drho.live());
  a.k = tp<T>(F.k.live());
  a.eps = tp<T>(F.eps.live());
  a.nut = tp<T>(F.nut.live());
  a.tag = F.tag.live();
  a.pid = F.pid.live();
  a.bufs = c->S.bufs;
  a.bidx = c->S.bidx;
  a.counters = c->S.counters;
  a.inj_key = c->S.inj_key;
  a.inj_idx = c->S.inj_idx;
  a.next_pid = c->S.next_pid;
  a.flags = c->S.flags;
  a.n = c->n_total;
  a.cap = c->cap;
  a.dim = c->P.dim;
  a.turb = c->P.turbulence;
  a.Cmu = c->P.Cmu;
  a.rho0 = c->P.rho0;
  a.c0 = c->P.c0;
  a.seed = c->P.seed;
  a.step = c->step;
  a.t = c->t;
  k_buffer_inject<T><<<1, kInjThreads, 0, c->stream>>>(a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_buffer_decide(sph_ctx* c, bool dry, uint32_t* dec_out, uint32_t* log,
                                int64_t pid_cap) {
  if (c->S.n_cand_cells == 0) return hipSuccess;
  BufArgs a = make_bufargs(c, dry, dec_out);
  a.log = log;
  a.pid_cap = pid_cap;
  k_buffer_decide<<<c->S.n_cand_cells, kWave, 0, c->stream>>>(a);
  return hipGetLastError();
}

hipError_t launch_buffer_forced(sph_ctx* c, const uint32_t* forced, uint32_t* log,
                                int64_t pid_cap) {
  if (c->n_total == 0) return hipSuccess;
  BufArgs a = make_bufargs(c, false, nullptr);
  a.forced = forced;
  a.log = log;
  a.pid_cap = pid_cap;
  k_buffer_forced<<<(int)((c->n_total + 255) / 256), 256, 0, c->stream>>>(a);
  return hipGetLastError();
}

// The injections of the decisions (the tag changes were applied with them).
hipError_t launch_buffer_inject(sph_ctx* c) {
  return c->P.precision == SPH_FP64 ? inject_impl<double>(c) : inject_impl<float>(c);
}

hipError_t launch_buffer_undo(sph_ctx* c, bool all_slots) {
  BufArgs a = make_bufargs(c, false, nullptr);
  if (all_slots) {
    if (c->n_total == 0) return hipSuccess;
    k_buffer_undo_all<<<(int)((c->n_total + 255) / 256), 256, 0, c->stream>>>(a);
  } else {
    if (c->S.n_cand_cells == 0) return hipSuccess;
    k_buffer_undo<<<c->S.n_cand_cells, kWave, 0, c->stream>>>(a);
  }
  return hipGetLastError();
}

}  // namespace sphx
