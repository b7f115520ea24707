// Cell-linked-list build (Sec. 2.4.1/2.4.3 of the paper: global cell list,
// rebuilt after deletion every advection step) as a counting sort on gfx950:
//   keys + per-cell histogram (integer atomics)  ->  exclusive scan  ->
//   scatter to the cell's slots  ->  placement of every particle at its rank
// inside the cell (ascending source index) with all its fields, emitting
// cell-relative positions in the pair precision.
// Also: particle upload / download and small fill kernels.
#include "sph_ctx.h"

namespace sphx {

namespace {

constexpr int kScanThreads = 1024;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

template <typename T>
__global__ void k_set_particles(int n, const double* __restrict__ x, const double* __restrict__ v,
                                const double* __restrict__ rho, const double* __restrict__ drho,
                                const double* __restrict__ kk, const double* __restrict__ ee,
                                const uint32_t* __restrict__ tag, const uint32_t* __restrict__ pid,
                                double* X0, double* X1, double* X2, T* V0, T* V1, T* V2,
                                double* R, T* DR, T* K, T* E, T* NT, uint32_t* TG, uint32_t* PD,
                                double Cmu, int turb) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  X0[i] = x[i];
  X1[i] = x[n + i];
  X2[i] = x[2 * n + i];
  V0[i] = (T)v[i];
  V1[i] = (T)v[n + i];
  V2[i] = (T)v[2 * n + i];
  R[i] = rho[i];
  DR[i] = drho ? (T)drho[i] : T(0);
  // nu_t of the stored (pair-precision) k and epsilon, as k_derive_nut
  const double k = (double)(T)((turb && kk) ? kk[i] : 0.0);
  const double e = (double)(T)((turb && ee) ? ee[i] : 0.0);
  K[i] = (T)k;
  E[i] = (T)e;
  NT[i] = (T)((turb && e > 0.0) ? Cmu * k * k / e : 0.0);
  TG[i] = tag[i];
  PD[i] = pid[i];
}

// Eddy viscosity of particles written in place: C_mu k^2 / epsilon from the
// stored k and epsilon (as k_set_particles computes it from its inputs).
template <typename T>
__global__ void k_derive_nut(int n, const T* __restrict__ K, const T* __restrict__ E,
                             T* __restrict__ NT, double Cmu, int turb) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double k = turb ? (double)K[i] : 0.0, e = turb ? (double)E[i] : 0.0;
  NT[i] = (T)((turb && e > 0.0) ? Cmu * k * k / e : 0.0);
}

template <typename T>
__global__ void k_get_particles(int n, double* x, double* v, double* rho, double* drho,
                                double* kk, double* ee, uint32_t* tag, uint32_t* pid,
                                const double* X0, const double* X1, const double* X2,
                                const T* V0, const T* V1, const T* V2, const double* R,
                                const T* DR, const T* K, const T* E, const uint32_t* TG,
                                const uint32_t* PD, int turb) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (x) { x[i] = X0[i]; x[n + i] = X1[i]; x[2 * n + i] = X2[i]; }
  if (v) { v[i] = (double)V0[i]; v[n + i] = (double)V1[i]; v[2 * n + i] = (double)V2[i]; }
  if (rho) rho[i] = R[i];
  if (drho) drho[i] = (double)DR[i];
  if (kk) kk[i] = turb ? (double)K[i] : 0.0;
  if (ee) ee[i] = turb ? (double)E[i] : 0.0;
  if (tag) tag[i] = TG[i];
  if (pid) pid[i] = PD[i];
}

// K1: cell id of every particle and a distinct slot inside its cell
// (cell_key_slot); particles tagged dead get key -1.  Block 0 also clears
// the buffer-update counters of this step.
constexpr int kKeysThreads = 1024;

template <int DIM>
__global__ __launch_bounds__(kKeysThreads) void k_cell_keys(
    int n, const double* __restrict__ x0, const double* __restrict__ x1,
    const double* __restrict__ x2, const uint32_t* __restrict__ tag, GridDev g,
    int32_t* __restrict__ key, int32_t* __restrict__ slot, int32_t* count,
    uint32_t* __restrict__ flags, int32_t* __restrict__ counters, int n_counters,
    const int32_t* __restrict__ ns) {
  if (ns) {
    if (ns[2]) return;
    n = ns[0];
  }
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x == 0)
    for (int q = threadIdx.x; q < n_counters; q += blockDim.x) counters[q] = 0;
  cell_key_slot<DIM>(i, n, x0, x1, x2, tag, g, key, slot, count, flags);
}

// K2 (grids of at most kSegScan cells): the whole exclusive scan in one
// workgroup.  Every wavefront scans one contiguous segment of the counts
// (coalesced, all loads in flight together), then the segment totals are
// combined; clears the counts for the next build.
constexpr int kSegThreads = 1024;
constexpr int kSegWaves = kSegThreads / kWave;
constexpr int kSegPer = 16;                                // counts per lane
constexpr int kSegScan = kSegWaves * kWave * kSegPer;      // 16384 cells

__global__ __launch_bounds__(kSegThreads) void k_scan_seg(int32_t* __restrict__ count, int nc,
                                                         int32_t* __restrict__ cell_start,
                                                         const int32_t* __restrict__ ns,
                                                         int32_t* __restrict__ counters) {
  if (ns && ns[2]) return;
  if (counters)   // the keys came with the post-update reduction: clear here
    for (int q = threadIdx.x; q < 1040; q += blockDim.x) counters[q] = 0;
  __shared__ int sm[kSegWaves];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const int per = (nc + kSegThreads - 1) / kSegThreads;   // <= kSegPer
  const int seg0 = w * per * kWave;
  int v[kSegPer];
#pragma unroll
  for (int q = 0; q < kSegPer; ++q) {
    const int idx = seg0 + q * kWave + lane;
    v[q] = (q < per && idx < nc) ? count[idx] : 0;
  }
  int run = 0;
#pragma unroll
  for (int q = 0; q < kSegPer; ++q) {
    const int inc = wave_incl_scan(v[q]);
    const int ex = run + inc - v[q];
    run += __builtin_amdgcn_readlane(inc, kWave - 1);
    v[q] = ex;
  }
  if (lane == 0) sm[w] = run;
  __syncthreads();
  int off = 0, total = 0;
#pragma unroll
  for (int q = 0; q < kSegWaves; ++q) {
    const int t = sm[q];
    off += q < w ? t : 0;
    total += t;
  }
#pragma unroll
  for (int q = 0; q < kSegPer; ++q) {
    const int idx = seg0 + q * kWave + lane;
    if (q < per && idx < nc) {
      cell_start[idx] = off + v[q];
      count[idx] = 0;
    }
  }
  if (threadIdx.x == 0) cell_start[nc] = total;
}

// K2: exclusive scan of the per-cell counts (reduce, scan of partials, apply).
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const int32_t* __restrict__ in,
                                                              int n, int32_t* __restrict__ part,
                                                              const int32_t* __restrict__ ns) {
  if (ns && ns[2]) return;
  __shared__ int sm[kScanThreads / kWave + 1];
  int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  int s = 0;
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) s += (base + q < n) ? in[base + q] : 0;
  int total;
  block_excl_scan(s, sm, &total);
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_parts(int32_t* __restrict__ part, int nb,
                                                             int32_t* __restrict__ out, int n,
                                                             const int32_t* __restrict__ ns,
                                                             int32_t* __restrict__ counters) {
  if (ns && ns[2]) return;
  if (counters)   // the keys came with the post-update reduction: clear here
    for (int q = threadIdx.x; q < 1040; q += blockDim.x) counters[q] = 0;
  __shared__ int sm[kScanThreads / kWave + 1];
  int base = threadIdx.x * kScanItems;
  int v[kScanItems];
  int s = 0;
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    v[q] = (base + q < nb) ? part[base + q] : 0;
    s += v[q];
  }
  int total;
  int off = block_excl_scan(s, sm, &total);
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    if (base + q < nb) part[base + q] = off;
    off += v[q];
  }
  if (threadIdx.x == 0) out[n] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(int32_t* __restrict__ in, int n,
                                                             const int32_t* __restrict__ part,
                                                             int32_t* __restrict__ out, int zero_in,
                                                             const int32_t* __restrict__ ns) {
  if (ns && ns[2]) return;
  __shared__ int sm[kScanThreads / kWave + 1];
  int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  int v[kScanItems];
  int s = 0;
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    v[q] = (base + q < n) ? in[base + q] : 0;
    s += v[q];
  }
  int total;
  int off = block_excl_scan(s, sm, &total) + part[blockIdx.x];
#pragma unroll
  for (int q = 0; q < kScanItems; ++q) {
    if (base + q < n) {
      out[base + q] = off;
      if (zero_in) in[base + q] = 0;
    }
    off += v[q];
  }
}

// K3a: scatter to cell-sorted positions (arbitrary order inside a cell).
// The entry is the source index with the particle's x quarter of its cell
// above it (bits 28-29; indices are below 2^26), so that entries order as
// the placement ranks them.
constexpr int kQuarterShift = 28;
__global__ void k_scatter(int n, const int32_t* __restrict__ key, const int32_t* __restrict__ slot,
                          const int32_t* __restrict__ cell_start, int32_t* __restrict__ perm,
                          const double* __restrict__ x0, GridDev g,
                          const int32_t* __restrict__ ns) {
  if (ns) {
    if (ns[2]) return;
    n = ns[0];
  }
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int k = key[i];
  if (k < 0) return;
  const int q = x_quarter(x0[i] - cell_centre(g.lo[0], k % g.n[0], g.cs), g.cs);
  perm[cell_start[k] + slot[i]] = i | (q << kQuarterShift);
}

// K3c: gather every field into cell order; cell-relative positions in T.
template <typename T, int DIM>
struct GatherArgs {
  const int32_t* perm;
  const int32_t* key;
  const int32_t* cell_start;
  int ncell;
  GridDev g;
  double mass, Vw;
  int turb;
  const double* x[3];
  double* xo[3];
  T* xro[3];
  const T* v[3];
  T* vo[3];
  const double* rho;
  double* rhoo;
  const T* drho;
  T* drhoo;
  const T *k, *eps, *nut;
  T *ko, *epso, *nuto;
  const uint32_t *tag, *pid;
  uint32_t *tago, *pido;
  T* volo;
  int32_t* cello;
  uint32_t* flags;
  const int32_t* ns;   // sizes on the device (prelaunched build), or NULL
  V4<T>* arec[3];      // advection records (written)
  int32_t* cell_q;     // starts of the x quarters 1-3 of each cell (written)
  float* xr32[3];      // FP32 copies of the cell-relative positions (or NULL)
};

// K3b: place every particle at its cell-ordered slot and copy its fields
// there.  Inside a cell the order is by quarter of the cell along x, then
// ascending source index (the previous, deterministic layout; new particles
// last): the rank of particle s is the number of particles of its cell in a
// lower quarter or in its quarter with a smaller source index, counted over
// the cell's (arbitrarily ordered) scatter slots.  The particle of rank 0
// also writes where the cell's quarters 1-3 start.
template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_place(int n_in, int n_out, GatherArgs<T, DIM> a) {
  if (a.ns) {
    if (a.ns[2]) return;
    n_in = a.ns[0];
    n_out = a.ns[1];
  }
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int total = a.cell_start[a.ncell];
  if (s == 0 && total != n_out) atomicOr(a.flags, kFlagCountMismatch);
  if (s >= n_in) return;
  // the source slot's fields load with its key, while the rank is found
  double xv[3];
  T vr[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    xv[k] = a.x[k][s];
    vr[k] = a.v[k][s];
  }
  const double r = a.rho[s];
  const T drho = a.drho[s];
  const uint32_t t = a.tag[s];
  const uint32_t pid = a.pid[s];
  T kt = T(0), et = T(0), nt = T(0);
  if (a.turb) {
    kt = a.k[s];
    et = a.eps[s];
    nt = a.nut[s];
  }
  const int c = a.key[s];
  if (c < 0) return;
  const int b = a.cell_start[c], e = a.cell_start[c + 1];
  int cc[3] = {c % a.g.n[0], (c / a.g.n[0]) % a.g.n[1], c / (a.g.n[0] * a.g.n[1])};
  const int me = s | (x_quarter(xv[0] - cell_centre(a.g.lo[0], cc[0], a.g.cs), a.g.cs)
                      << kQuarterShift);
  int rank = 0, n1 = 0, n2 = 0, n3 = 0;   // n_k: members in quarters below k
  for (int q = b; q < e; ++q) {
    const int pq = a.perm[q];
    n1 += pq < (1 << kQuarterShift) ? 1 : 0;
    n2 += pq < (2 << kQuarterShift) ? 1 : 0;
    n3 += pq < (3 << kQuarterShift) ? 1 : 0;
    rank += pq < me ? 1 : 0;
  }
  if (rank == 0)
    *reinterpret_cast<int4*>(a.cell_q + 4 * (int64_t)c) = int4{b + n1, b + n2, b + n3, e};
  const int d = b + rank;
  if (d >= n_out) return;
  T xr[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    a.xo[k][d] = xv[k];
    double org = (k < DIM) ? cell_centre(a.g.lo[k], cc[k], a.g.cs) : 0.0;
    xr[k] = (T)(xv[k] - org);
    a.xro[k][d] = xr[k];
    if (a.xr32[0]) a.xr32[k][d] = (float)(xv[k] - org);
    a.vo[k][d] = vr[k];
  }
  a.rhoo[d] = r;
  a.drhoo[d] = drho;
  a.tago[d] = t;
  a.pido[d] = pid;
  const bool wall = tag_kind(t) == kWall;
  const T vol = (T)(wall ? a.Vw : a.mass / r);
  a.volo[d] = vol;
  a.cello[d] = c;
  if (a.turb) {
    a.ko[d] = kt;
    a.epso[d] = et;
    a.nuto[d] = nt;
  }
  write_arec<T, DIM>(a.arec, d, xr, vr, wall ? -vol : vol, nt, kt, et, a.turb != 0);
}

template <typename T>
T* tp(void* p) { return static_cast<T*>(p); }

// n_in / n_out: particles before / after the build; with ns (device
// {n_in, n_out, skip}) they are upper bounds that size the grids.
template <typename T, int DIM>
hipError_t build_cells_impl(sph_ctx* c, int64_t n_in, int64_t n_out, const int32_t* ns,
                            bool keys_done) {
  hipStream_t st = c->stream;
  Fields& F = c->F;
  Scratch& S = c->S;
  const GridDev& g = c->grid;
  const int nc = g.ncell;
  // the counts are cleared by the scan of the previous build (and at create)
  int32_t* clear = keys_done ? S.counters : nullptr;
  if (keys_done) {
    // keys, slots and counts came with the post-update reduction
  } else if (n_in > 0) {
    k_cell_keys<DIM><<<(int)((n_in + kKeysThreads - 1) / kKeysThreads), kKeysThreads, 0, st>>>(
        (int)n_in, F.x[0].live(), F.x[1].live(), F.x[2].live(), F.tag.live(), g, S.key, S.slot,
        S.count, S.flags, S.counters, 1040, ns);
  } else {
    k_fill_i32<<<(1040 + 255) / 256, 256, 0, st>>>(S.counters, 1040, 0);
  }
  if (nc <= kSegScan) {
    k_scan_seg<<<1, kSegThreads, 0, st>>>(S.count, nc, S.cell_start, ns, clear);
  } else {
    int nb = (nc + kScanTile - 1) / kScanTile;
    k_scan_reduce<<<nb, kScanThreads, 0, st>>>(S.count, nc, S.block_sums, ns);
    k_scan_parts<<<1, kScanThreads, 0, st>>>(S.block_sums, nb, S.cell_start, nc, ns, clear);
    k_scan_apply<<<nb, kScanThreads, 0, st>>>(S.count, nc, S.block_sums, S.cell_start, 1, ns);
  }
  if (n_in > 0)
    k_scatter<<<(int)((n_in + 255) / 256), 256, 0, st>>>(
        (int)n_in, S.key, S.slot, S.cell_start, S.perm, F.x[0].live(), g, ns);
  GatherArgs<T, DIM> a;
  a.perm = S.perm;
  a.key = S.key;
  a.cell_start = S.cell_start;
  a.ncell = nc;
  a.g = g;
  double Vw = c->P.dim == 2 ? c->P.dp * c->P.dp : c->P.dp * c->P.dp * c->P.dp;
  a.mass = c->P.rho0 * Vw;
  a.Vw = Vw;
  a.turb = c->P.turbulence;
  for (int k = 0; k < 3; ++k) {
    a.x[k] = F.x[k].live();
    a.xo[k] = F.x[k].other();
    a.xro[k] = tp<T>(F.xr[k].other());
    a.v[k] = tp<T>(F.v[k].live());
    a.vo[k] = tp<T>(F.v[k].other());
  }
  a.rho = F.rho.live();
  a.rhoo = F.rho.other();
  a.drho = tp<T>(F.drho.live());
  a.drhoo = tp<T>(F.drho.other());
  a.k = tp<T>(F.k.live());
  a.eps = tp<T>(F.eps.live());
  a.nut = tp<T>(F.nut.live());
  a.ko = tp<T>(F.k.other());
  a.epso = tp<T>(F.eps.other());
  a.nuto = tp<T>(F.nut.other());
  a.tag = F.tag.live();
  a.pid = F.pid.live();
  a.tago = F.tag.other();
  a.pido = F.pid.other();
  a.volo = tp<T>(F.vol.a[0]);
  a.cello = F.cell;
  a.flags = S.flags;
  a.ns = ns;
  for (int k = 0; k < 3; ++k) a.arec[k] = static_cast<V4<T>*>(F.arec[k]);
  a.cell_q = S.cell_q;
  for (int k = 0; k < 3; ++k) a.xr32[k] = F.xr32[k];
  k_place<T, DIM><<<(int)((n_in + 255) / 256) + (n_in == 0), 256, 0, st>>>((int)n_in, (int)n_out, a);
  for (int k = 0; k < 3; ++k) {
    F.x[k].flip();
    F.xr[k].cur = F.x[k].cur;
    F.v[k].flip();
  }
  F.rho.flip();
  F.drho.flip();
  F.tag.flip();
  F.pid.flip();
  if (c->P.turbulence) {
    F.k.flip();
    F.eps.flip();
    F.nut.flip();
  }
  F.p.cur = 0;
  F.vol.cur = 0;
  return hipGetLastError();
}

template <typename T>
hipError_t set_impl(sph_ctx* c, int64_t n, const sph_particles* s) {
  Fields& F = c->F;
  int turb = c->P.turbulence;
  k_set_particles<T><<<(int)((n + 255) / 256) + (n == 0), 256, 0, c->stream>>>(
      (int)n, s->x, s->v, s->rho, s->drho, s->k, s->eps, s->tag, s->pid, F.x[0].live(),
      F.x[1].live(), F.x[2].live(), tp<T>(F.v[0].live()), tp<T>(F.v[1].live()),
      tp<T>(F.v[2].live()), F.rho.live(), tp<T>(F.drho.live()), tp<T>(F.k.live()),
      tp<T>(F.eps.live()), tp<T>(F.nut.live()), F.tag.live(), F.pid.live(), c->P.Cmu, turb);
  return hipGetLastError();
}

template <typename T>
hipError_t get_impl(sph_ctx* c, const sph_particles* d) {
  Fields& F = c->F;
  int64_t n = c->n_total;
  k_get_particles<T><<<(int)((n + 255) / 256) + (n == 0), 256, 0, c->stream>>>(
      (int)n, d->x, d->v, d->rho, d->drho, d->k, d->eps, d->tag, d->pid, F.x[0].live(),
      F.x[1].live(), F.x[2].live(), tp<T>(F.v[0].live()), tp<T>(F.v[1].live()),
      tp<T>(F.v[2].live()), F.rho.live(), tp<T>(F.drho.live()), tp<T>(F.k.live()),
      tp<T>(F.eps.live()), F.tag.live(), F.pid.live(), c->P.turbulence);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_scan_excl_part(sph_ctx* c, const int32_t* in, int n, int32_t* out,
                                 int32_t* part) {
  const int nb = (n + kScanTile - 1) / kScanTile + (n == 0);
  if (nb > kScanTile) return hipErrorInvalidValue;
  k_scan_reduce<<<nb, kScanThreads, 0, c->stream>>>(in, n, part, nullptr);
  k_scan_parts<<<1, kScanThreads, 0, c->stream>>>(part, nb, out, n, nullptr, nullptr);
  k_scan_apply<<<nb, kScanThreads, 0, c->stream>>>(const_cast<int32_t*>(in), n, part, out, 0,
                                                    nullptr);
  return hipGetLastError();
}

hipError_t launch_scan_excl(sph_ctx* c, const int32_t* in, int n, int32_t* out) {
  return launch_scan_excl_part(c, in, n, out, c->S.block_sums);
}

hipError_t launch_zero_i32(sph_ctx* c, int32_t* p, int64_t n) {
  if (n <= 0) return hipSuccess;
  k_fill_i32<<<(int)((n + 255) / 256), 256, 0, c->stream>>>(p, n, 0);
  return hipGetLastError();
}

hipError_t launch_set_particles(sph_ctx* c, int64_t n, const sph_particles* src) {
  return c->P.precision == SPH_FP64 ? set_impl<double>(c, n, src) : set_impl<float>(c, n, src);
}

hipError_t launch_derive_nut(sph_ctx* c, int64_t n) {
  Fields& F = c->F;
  const int nb = (int)((n + 255) / 256) + (n == 0);
  if (c->P.precision == SPH_FP64)
    k_derive_nut<double><<<nb, 256, 0, c->stream>>>((int)n, tp<double>(F.k.live()),
                                                     tp<double>(F.eps.live()),
                                                     tp<double>(F.nut.live()), c->P.Cmu,
                                                     c->P.turbulence);
  else
    k_derive_nut<float><<<nb, 256, 0, c->stream>>>((int)n, tp<float>(F.k.live()),
                                                    tp<float>(F.eps.live()),
                                                    tp<float>(F.nut.live()), c->P.Cmu,
                                                    c->P.turbulence);
  return hipGetLastError();
}

hipError_t launch_get_particles(sph_ctx* c, const sph_particles* dst) {
  return c->P.precision == SPH_FP64 ? get_impl<double>(c, dst) : get_impl<float>(c, dst);
}

hipError_t launch_build_cells(sph_ctx* c, int64_t n_in, int64_t n_out, const int32_t* ns,
                              bool keys_done) {
  if (c->P.precision == SPH_FP64)
    return c->P.dim == 2 ? build_cells_impl<double, 2>(c, n_in, n_out, ns, keys_done)
                         : build_cells_impl<double, 3>(c, n_in, n_out, ns, keys_done);
  return c->P.dim == 2 ? build_cells_impl<float, 2>(c, n_in, n_out, ns, keys_done)
                       : build_cells_impl<float, 3>(c, n_in, n_out, ns, keys_done);
}

}  // namespace sphx
