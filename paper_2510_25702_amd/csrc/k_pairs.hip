// Neighbour passes of the SPH step on gfx950 (Sec. 2.2 of the paper).
//
// Layout: every field is a structure-of-arrays in cell order (built by
// k_cells.hip).  A team of L lanes (one to eight, by problem size) owns one
// particle i.  The correction pass scans the 3^dim cells around i's build
// cell (in each cell row the three cells are one contiguous index range)
// and writes the step's neighbour list; the advection, pressure and
// continuity passes walk that list and gather packed 16-byte records of
// their neighbours.  Pair arithmetic runs in T (float in FP32-mixed mode,
// double in FP64 mode) on cell-relative positions; densities, positions and
// the inversion of the correction matrix stay in FP64.  Every particle sums
// its own neighbours (gather form) and the team reduces in a fixed order:
// no floating-point atomics, results are deterministic.
#include <mutex>

#include "sph_pairs.h"

namespace sphx {

// Device memory of sph_neighbors_noalloc, for callers that cannot allocate:
// per-particle neighbour counts and the partial sums of their scan.  One
// copy per device, held until the process ends and shared by every call on
// that device.  Host code uses its device address (noalloc_scratch_init),
// never this name.
constexpr int64_t kNoAllocMaxN = SPH_NOALLOC_MAX_PARTICLES;
constexpr int64_t kNoAllocParts = 4096;   // scan tiles of 4096 counts
static __device__ __align__(256) int32_t scratch[kNoAllocMaxN + kNoAllocParts];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int32_t* g_scratch_dev[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_dev[device] = static_cast<int32_t*>(p);
  return hipSuccess;
}

namespace {

// ---------------------------------------------------------------------------
// K5: correction matrix, Eq. (equ-B-matrix): A_i = -sum_j V_j r_ij (x) gradW_ij,
// plus mirror images across every buffer's open face (Sec. 3.3) for
// obc_mode >= 3, B_i = A_i^-1 in FP64 with a singularity guard.
// ---------------------------------------------------------------------------
template <typename T>
struct CorrArgs {
  const double* x[3];
  const BufDev* bufs;
  T* B[6];
  uint32_t* flags;
  int mirror;
  const V4<T>* arec[2];   // the cell build's advection records (the list moment)
};

// The 3D correction runs as two kernels: the stencil scan writes the list
// only (MOMENT false), then the kernel without BUILD takes the moment and B
// over the list it wrote (~100 entries instead of ~1000 candidates whose
// terms a wavefront evaluated on nearly every batch).  2D scans ~100
// candidates against ~25 entries and keeps one kernel.  The moment walk
// (REC) reads the list the way the other list passes do: deep batches of
// the advection records written by the cell build, the next batch's entries
// loading under the current records.  In sph_advance's 3D laminar steps the
// advection pass forms B in its own walk instead (advection_body, MOM).
template <int DIM>
constexpr bool split_correction() {
  return DIM == 3;
}

// One pair's term of the moment A_i = -sum_j V_j f_ij r_ij (x) r_ij
// (symmetric, packed xx xy xz yy yz zz), Eq. (equ-B-matrix).
template <typename T, int DIM>
__device__ __forceinline__ void moment_pair(T (&A)[6], const T r[3], T r2, T Vj,
                                            const Consts<T>& C) {
  const T f = dw_over_r<T>(pair_dist(r2), C.inv_h_t, C.kf_t);
  const T Vf = Vj * f;
  A[0] -= Vf * r[0] * r[0];
  A[1] -= Vf * r[0] * r[1];
  A[3] -= Vf * r[1] * r[1];
  if (DIM == 3) {
    A[2] -= Vf * r[0] * r[2];
    A[4] -= Vf * r[1] * r[2];
    A[5] -= Vf * r[2] * r[2];
  }
}

// The end of particle i's moment after its pair walk (every lane of the
// team): the terms of the mirror images at the open faces (obc_mode >= 3,
// Sec. 3.3), the team sum, B_i = A_i^-1 in FP64 with the singularity guard.
// Lane 0 writes B_i and returns it in Bt.
template <typename T, int DIM, int L>
__device__ __forceinline__ void moment_finish(int i, int lane, const PairCtx<T>& pc,
                                              const Consts<T>& C, const CorrArgs<T>& a,
                                              T (&A)[6], T (&Bt)[6]) {
  if (a.mirror) {
    const double xi0 = a.x[0][i], xi1 = a.x[1][i], xi2 = a.x[2][i];
    const double twoh = 2.0 * C.h;
    for (int q = 0; q < C.nbuf; ++q) {
      const BufDev& b = a.bufs[q];
      double yi[3];
      to_local(b, xi0, xi1, xi2, yi);
      if (!(yi[0] >= 0.0 && yi[0] < twoh)) continue;
      // the buffer's particles lie within its transverse half-widths, and
      // the mirror keeps their transverse coordinates: beyond hw + 2h (a
      // little more, for the pair test's rounding) no image is within 2h.
      // The face plane is unbounded, so without this test every particle
      // within 2h of it searched the stencil around its image (on the 3D
      // mixer, with its four tangential inlets: 0.71 of 1.59 ms of the pass)
      const double reach = twoh * (1.0 + 1e-5);
      if (!(fabs(yi[1]) < b.hw[0] + reach) || (DIM == 3 && !(fabs(yi[2]) < b.hw[1] + reach)))
        continue;
      const double tt = 2.0 * yi[0];
      const double m[3] = {xi0 - tt * b.frame[0], xi1 - tt * b.frame[1], xi2 - tt * b.frame[2]};
      int cm[3] = {0, 0, 0};
      bool ok = true;
      for (int k = 0; k < DIM; ++k) {
        cm[k] = cell_coord(m[k], C.grid.lo[k], C.grid.cs);
        if (cm[k] < 1 || cm[k] > C.grid.n[k] - 2) ok = false;
      }
      if (!ok) {
        atomicOr(a.flags, kFlagOutOfGrid);
        continue;
      }
      constexpr int zr = DIM == 3 ? 1 : 0;
      for (int dz = -zr; dz <= zr; ++dz)
        for (int dy = -1; dy <= 1; ++dy) {
          const int base = ((cm[2] + dz) * pc.ny + (cm[1] + dy)) * pc.nx + cm[0];
          const int j0 = pc.cs[base - 1], j3 = pc.cs[base + 2];
          for (int j = j0 + lane; j < j3; j += L) {
            if (!is_real(pc.tag[j])) continue;
            double yj[3];
            const double xj0 = a.x[0][j], xj1 = a.x[1][j], xj2 = a.x[2][j];
            to_local(b, xj0, xj1, xj2, yj);
            if (!(yj[0] >= 0.0) || !contained(DIM, b, yj)) continue;
            const double tj = 2.0 * yj[0];
            const T r[3] = {(T)(xi0 - (xj0 - tj * b.frame[0])),
                            (T)(xi1 - (xj1 - tj * b.frame[1])),
                            (T)(DIM == 3 ? xi2 - (xj2 - tj * b.frame[2]) : 0.0)};
            const T r2 = DIM == 3 ? (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]
                                  : r[0] * r[0] + r[1] * r[1];
            if (r2 < pc.rc2) moment_pair<T, DIM>(A, r, r2, pc.vol[j], C);
          }
        }
    }
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) A[k] = team_sum<L>(A[k]);
  if (lane != 0) return;
  double Ad[6] = {(double)A[0], (double)A[1], (double)A[2],
                  (double)A[3], (double)A[4], (double)A[5]};
  double Bd[6];
  invert_sym<DIM>(Ad, Bd);
#pragma unroll
  for (int k = 0; k < 6; ++k) Bt[k] = (DIM == 2 && (k == 2 || k == 4 || k == 5)) ? T(0) : (T)Bd[k];
  a.B[0][i] = Bt[0];
  a.B[1][i] = Bt[1];
  a.B[3][i] = Bt[3];
  if (DIM == 3) {
    a.B[2][i] = Bt[2];
    a.B[4][i] = Bt[4];
    a.B[5][i] = Bt[5];
  }
}

template <typename T, int DIM, int L, bool BUILD, bool MOMENT = true, bool REC = false>
__device__ __forceinline__ int correction_body(int i, int lane, int n, const PairCtx<T>& pc,
                                               const Consts<T>& C, const CorrArgs<T>& a,
                                               const NbrOut<T>& nb) {
  if (i >= n) return 0;
  int m_pairs = 0;
  constexpr int NR = 2;
  ListHead<rec_unroll<T, DIM, L, NR>()> head{};
  if constexpr (REC) head = list_head<T, DIM, L, NR>(pc, i, lane);
  const uint32_t ti = pc.tag[i];
  if (BUILD) build_begin<T, DIM>(pc, i, lane, nb);
  if (BUILD && !MOMENT) {
    if (is_real(ti)) {
      const T xi[3] = {pc.xr[0][i], pc.xr[1][i], DIM == 3 ? pc.xr[2][i] : T(0)};
      scan_build<T, DIM, L, 0, true>(pc, i, lane, xi, nb, [](int, const T*, T, T) {});
    }
    return m_pairs;
  }
  if (!is_real(ti)) {
    if (lane == 0) {
      a.B[0][i] = T(1); a.B[1][i] = T(0); a.B[3][i] = T(1);
      if (DIM == 3) { a.B[2][i] = T(0); a.B[4][i] = T(0); a.B[5][i] = T(1); }
    }
    return m_pairs;
  }
  const T xi[3] = {pc.xr[0][i], pc.xr[1][i], DIM == 3 ? pc.xr[2][i] : T(0)};
  T A[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
  auto pair = [&](int j, const T r[3], T r2) {
    moment_pair<T, DIM>(A, r, r2, pc.vol[j], C);
    ++m_pairs;
  };
  auto pair_v = [&](int, const T r[3], T r2, T vj) {   // V_j loaded with the positions
    moment_pair<T, DIM>(A, r, r2, vj, C);
    ++m_pairs;
  };
  if (BUILD) {
    scan_build<T, DIM, L>(pc, i, lane, xi, nb, pair_v);
  } else if (REC) {
    // V_j from the record, its sign (a wall) dropped
    for_neighbors_rec<T, DIM, L, NR>(pc, i, lane, xi, a.arec, head,
                                     [&](int, const T r[3], T r2, const auto& q) {
                                       moment_pair<T, DIM>(A, r, r2, fabs(q[1].c), C);
                                       ++m_pairs;
                                     });
  } else {
    for_neighbors<T, DIM, L>(pc, i, lane, xi, pair);
  }
  T Bt[6];
  moment_finish<T, DIM, L>(i, lane, pc, C, a, A, Bt);
  return m_pairs;
}

// Wavefronts per SIMD that the FP32 3D list-only scan is compiled for (1:
// the compiler's choice, 67 registers and seven wavefronts).  8 fits 64
// registers with 12 bytes of scratch per lane: the mixer's correction 4315
// -> 4240 us, left out to keep every kernel free of scratch memory.
#ifndef SPHX_SCAN_WAVES
#define SPHX_SCAN_WAVES 1
#endif
template <typename T, int DIM, int L, bool BUILD>
constexpr int scan_waves() {
  return (BUILD && DIM == 3 && sizeof(T) == 4) ? SPHX_SCAN_WAVES : 1;
}

template <typename T, int DIM, int L, bool BUILD, bool MOMENT = true, bool REC = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(
    (!MOMENT) ? scan_waves<T, DIM, L, BUILD>() : 1))) void k_correction(int n, PairCtx<T> pc, Consts<T> C, CorrArgs<T> a,
                                                    NbrOut<T> nb, const int32_t* __restrict__ ns) {
  if (ns) {   // sizes on the device: the build of this state was prelaunched
    if (ns[2]) return;
    n = ns[1];
  }
  const int g = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (BUILD && g == 0) {
    nb.stale[0] = 0;
    nb.stale[1] = 0;
    // whether this pass lists by the relative-motion radius, for the passes' check of it
    nb.lrad[1] = (nb.tight && nb.lrad[0] > 0.0) ? 1.0 : 0.0;
  }
  constexpr int KS = BUILD ? list_stage<DIM, L>() : 0;
  __shared__ uint32_t stage[KS > 0 ? (256 / L) * KS : 1];
  nb.kstage = KS;
  nb.stage = KS > 0 ? stage + (threadIdx.x / L) * KS : nullptr;
  constexpr int PQ = (BUILD && MOMENT) ? pair_queue<T, DIM>() : 0;
  __shared__ V4<T> pqueue[PQ > 0 ? PQ * 256 : 1];
  nb.queue = PQ > 0 ? pqueue + (threadIdx.x / kWave) * (PQ * kWave) : nullptr;
  const int m = correction_body<T, DIM, L, BUILD, MOMENT, REC>(g / L, g % L, n, pc, C, a, nb);
  count_pairs(pc.pairs, m);
}

// ---------------------------------------------------------------------------
// K6: advection-level pass.  ARD viscous acceleration, Eqs.
// (eq-discretize-momentum-ARD2/-ARD-viscosity); RANS: velocity gradient,
// Eq. (velo-grad-equ), k / epsilon diffusion and sources, Eqs.
// (k-/epsilon-discretized-equ), explicit update over dt_adv, floors and
// free-stream values; then the first half density update of the first
// acoustic sub-step and its pressure / volume.
// ---------------------------------------------------------------------------
template <typename T>
struct AdvArgs {
  const T* v[3];
  double* rho;
  const T* drho;
  const T* B[6];
  const T *k, *eps, *nut;
  T *ko, *epso, *nuto;
  T* anu[3];
  T *p_out, *vol_out;
  const BufDev* bufs;
  const int32_t* bidx;
  double dt_adv, half_dt;
  int rates_only;
  double *o_anu, *o_gradv, *o_dk, *o_deps;
  int64_t n_out;
  V4<T>* prec[3];   // pressure records of sub-step 0 (written)
  const V4<T>* arec[3];   // advection records (cell build)
  int tvf;                // transport-velocity shift summed (uniform switch)
  double tvf_c;           // -2 tvf_alpha h^2
  double two_h;           // buffer particles within 2h of the box ends: no shift
  const double* x[3];     // FP64 positions (buffer particles' local frame)
  T* shift[3];            // the shift of fluid particles (written)
  double* o_shift;        // rates output [3][n_out]
  CorrArgs<T> cor;        // the correction's operands (MOM: B formed in this pass)
};

// MOM (3D laminar list passes): the pass also forms the correction matrix
// B_i over the same walk of the list -- the moment terms of each pair, then
// the mirror images, the team sum and the guarded FP64 inverse, the
// correction kernel's own code in its order, so B is the same bit for bit
// -- instead of a separate walk of the list by the correction; B is first
// needed by this pass's pressure record.
template <typename T, int DIM, int TURB, int L, bool MOM = false>
__device__ __forceinline__ int advection_body(int i, int lane, int n, const PairCtx<T>& pc,
                                              const Consts<T>& C, const AdvArgs<T>& a) {
  if (i >= n) return 0;
  int m_pairs = 0;
  // the tag, the position and the head of the list load together
  constexpr int NR = (DIM == 3 && TURB) ? 3 : 2;   // record vectors
  const uint32_t ti = pc.tag[i];
  const auto h = list_head<T, DIM, L, NR>(pc, i, lane);
  const T xi[3] = {pc.xr[0][i], pc.xr[1][i], DIM == 3 ? pc.xr[2][i] : T(0)};
  if (!is_real(ti)) {
    if (a.rates_only && lane == 0) {   // walls and dead slots: zero rates
      for (int k = 0; k < 3; ++k) {
        if (a.o_anu) a.o_anu[(int64_t)k * a.n_out + i] = 0.0;
        if (a.o_shift) a.o_shift[(int64_t)k * a.n_out + i] = 0.0;
      }
      if (TURB) {
        if (a.o_dk) a.o_dk[i] = 0.0;
        if (a.o_deps) a.o_deps[i] = 0.0;
        if (a.o_gradv)
          for (int p = 0; p < 9; ++p) a.o_gradv[(int64_t)p * a.n_out + i] = 0.0;
      }
    }
    if (!a.rates_only && lane == 0) {
      if (MOM) {   // as the correction: the identity for walls and dead slots
        a.cor.B[0][i] = T(1); a.cor.B[1][i] = T(0); a.cor.B[3][i] = T(1);
        a.cor.B[2][i] = T(0); a.cor.B[4][i] = T(0); a.cor.B[5][i] = T(1);
      }
      for (int k = 0; k < 3; ++k) a.anu[k][i] = T(0);
      a.p_out[i] = T(0);
      a.vol_out[i] = (T)C.Vw;
      if (TURB) { a.ko[i] = T(0); a.epso[i] = T(0); a.nuto[i] = T(0); }
      const T Iw[6] = {T(1), T(0), T(0), T(1), T(0), T(1)};
      write_prec<T, DIM>(a.prec, i, xi, T(0), -(T)C.Vw, Iw);
    }
    return m_pairs;
  }
  const T vi[3] = {a.v[0][i], a.v[1][i], DIM == 3 ? a.v[2][i] : T(0)};
  const double rho_i = a.rho[i];
  const T nut_i = TURB ? a.nut[i] : T(0);
  const T mu_i = C.rho0_t * ((T)C.nu_l + nut_i);
  T av[3] = {T(0), T(0), T(0)};
  T G[9] = {T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
  T Bi[6];
  T ki = T(0), ei = T(0), Dk_i = T(0), De_i = T(0), dfk = T(0), dfe = T(0);
  T sh[3] = {T(0), T(0), T(0)};   // sum_j V_j grad_i W_ij (transport velocity)
  T Am[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};   // the moment (MOM)
  if (TURB) {
    load_B<T, DIM>(a.B, i, Bi);   // the velocity gradient's correction
    ki = a.k[i];
    ei = a.eps[i];
    Dk_i = (T)C.nu_l + nut_i / (T)C.sigma_k;
    De_i = (T)C.nu_l + nut_i / (T)C.sigma_eps;
  }
  // B for the pressure record (laminar), the continuity rate and the buffer
  // index, needed after the sum: issued before the walk by wide teams,
  // after the sum by narrow ones
  T drho_i = T(0);
  int qb = -1;
  auto load_update = [&]() {
    if (!TURB && !a.rates_only && !MOM) load_B<T, DIM>(a.B, i, Bi);
    if (!a.rates_only) drho_i = a.drho[i];
    if (TURB && tag_kind(ti) == kBuffer) qb = a.bidx[tag_bid(ti)];
  };
  constexpr bool early = hoist_epilogue<L>();
  if (early) load_update();
  for_neighbors_rec<T, DIM, L, NR>(pc, i, lane, xi, a.arec, h,
                                   [&](int j, const T r[3], T r2, const V4<T>* q) {
    ++m_pairs;
    const T rr = pair_dist(r2);
    const T f = dw_over_r<T>(rr, C.inv_h_t, C.kf_t);
    T vj[3], volw, nut_rj, k_j, eps_j;
    if (DIM == 2) {
      vj[0] = q[0].c; vj[1] = q[0].d; vj[2] = T(0);
      volw = q[1].a; nut_rj = q[1].b; k_j = q[1].c; eps_j = q[1].d;
    } else {
      vj[0] = q[0].d; vj[1] = q[1].a; vj[2] = q[1].b;
      volw = q[1].c; nut_rj = q[1].d;
      k_j = TURB ? q[2].a : T(0);
      eps_j = TURB ? q[2].b : T(0);
    }
    const bool wall = volw < T(0);
    const T Vj = wall ? -volw : volw;
    if constexpr (MOM) moment_pair<T, DIM>(Am, r, r2, Vj, C);
    // no-slip dummy wall: antisymmetric velocity, same viscosity as i
    T vij[3];
    if (wall) {
      vij[0] = T(2) * vi[0]; vij[1] = T(2) * vi[1]; vij[2] = T(2) * vi[2];
    } else {
      vij[0] = vi[0] - vj[0];
      vij[1] = vi[1] - vj[1];
      vij[2] = DIM == 3 ? vi[2] - vj[2] : T(0);
    }
    T mu_ad;
    if (TURB) {
      const T nut_j = wall ? nut_i : nut_rj;
      const T mu_j = C.rho0_t * ((T)C.nu_l + nut_j);
      const T mu_h = T(2) * mu_i * mu_j / (mu_i + mu_j);
      // ARD limiter: beta = min(eta max(v_ij . e_ij, 0), c0), e_ij from i to j
      T beta = T(0);
      if (rr > T(0)) {
        const T ve = -(vij[0] * r[0] + vij[1] * r[1] + vij[2] * r[2]) / rr;
        beta = fmin(C.eta_t * fmax(ve, T(0)), C.c0_t);
      }
      mu_ad = fmax(mu_h, C.mu_R_t * beta);
    } else {
      mu_ad = mu_i;
    }
    const T s = mu_ad * f * Vj;
    av[0] += s * vij[0];
    av[1] += s * vij[1];
    av[2] += s * vij[2];
    if (a.tvf) {
      const T fv = f * Vj;
#pragma unroll
      for (int k = 0; k < DIM; ++k) sh[k] += fv * r[k];
    }
    if (TURB) {
      const T gW[3] = {f * r[0], f * r[1], f * r[2]};
      T BgW[3];
      symv<T, DIM>(Bi, gW, BgW);
#pragma unroll
      for (int p = 0; p < DIM; ++p)
#pragma unroll
        for (int q = 0; q < DIM; ++q) G[3 * p + q] -= Vj * vij[p] * BgW[q];
      if (!wall) {
        const T nut_j = nut_rj;
        const T Dk_j = (T)C.nu_l + nut_j / (T)C.sigma_k;
        const T De_j = (T)C.nu_l + nut_j / (T)C.sigma_eps;
        dfk += T(2) * Dk_i * Dk_j / (Dk_i + Dk_j) * (ki - k_j) * f * Vj;
        dfe += T(2) * De_i * De_j / (De_i + De_j) * (ei - eps_j) * f * Vj;
      }
    }
  });
  if constexpr (MOM) moment_finish<T, DIM, L>(i, lane, pc, C, a.cor, Am, Bi);
#pragma unroll
  for (int k = 0; k < 3; ++k) av[k] = team_sum<L>(av[k]);
  if (a.tvf) {
#pragma unroll
    for (int k = 0; k < DIM; ++k) sh[k] = team_sum<L>(sh[k]);
  }
  if (TURB) {
#pragma unroll
    for (int k = 0; k < 9; ++k) G[k] = team_sum<L>(G[k]);
    dfk = team_sum<L>(dfk);
    dfe = team_sum<L>(dfe);
  }
  if (lane != 0) return m_pairs;
  if (!early) load_update();
  const double two_over_rho = 2.0 / rho_i;
  double anu_d[3] = {two_over_rho * (double)av[0], two_over_rho * (double)av[1],
                     two_over_rho * (double)av[2]};
  double k_new = 0.0, e_new = 0.0, nut_new = 0.0;
  if (TURB) {
    double diff_k = two_over_rho * (double)dfk, diff_e = two_over_rho * (double)dfe;
    double dd = 0.0, tr = 0.0;
    for (int p = 0; p < DIM; ++p) {
      tr += (double)G[3 * p + p];
      for (int q = 0; q < DIM; ++q)
        dd += ((double)G[3 * p + q] + (double)G[3 * q + p]) * (double)G[3 * p + q];
    }
    const double kd = (double)ki, ed = (double)ei;
    const double Gk = (double)nut_i * dd - (2.0 / 3.0) * kd * tr;
    const double dk = Gk - ed + diff_k;
    const double de = C.C1 * (ed / kd) * Gk - C.C2 * ed * ed / kd + diff_e;
    if (a.rates_only) {
      if (a.o_dk) a.o_dk[i] = dk;
      if (a.o_deps) a.o_deps[i] = de;
      if (a.o_gradv)
        for (int p = 0; p < 9; ++p) a.o_gradv[(int64_t)p * a.n_out + i] = (double)G[p];
    } else {
      k_new = fmax(kd + a.dt_adv * dk, C.k_floor);
      e_new = fmax(ed + a.dt_adv * de, C.eps_floor);
      if (qb >= 0 && a.bufs[qb].turb_mode == kTurbFreestream) {
        k_new = a.bufs[qb].k_bc;
        e_new = a.bufs[qb].eps_bc;
      }
      nut_new = C.Cmu * k_new * k_new / e_new;
    }
  }
  if (a.tvf) {   // particles that move with the flow: fluid, extrapolating buffers
    double d[3] = {0.0, 0.0, 0.0};
    const int qs = tag_kind(ti) == kBuffer ? a.bidx[tag_bid(ti)] : -1;
    const BufDev* bq = qs >= 0 ? &a.bufs[qs] : nullptr;   // unknown id: no shift
    if (tag_kind(ti) == kFluid || (bq && bq->vel_mode == kVelExtrapolate)) {
      for (int k = 0; k < DIM; ++k) d[k] = a.tvf_c * (double)sh[k];
      if (bq) {   // along the open face only (normal n_b removed), none near the ends
        const double r0[3] = {a.x[0][i] - bq->origin[0], a.x[1][i] - bq->origin[1],
                              DIM == 3 ? a.x[2][i] - bq->origin[2] : 0.0 - bq->origin[2]};
        const double* fr = bq->frame;
        const double y1 = (fr[3] * r0[0] + fr[4] * r0[1]) + fr[5] * r0[2];
        const double y2 = (fr[6] * r0[0] + fr[7] * r0[1]) + fr[8] * r0[2];
        const bool end = fabs(y1) > bq->hw[0] - a.two_h ||
                         (DIM == 3 && fabs(y2) > bq->hw[1] - a.two_h);
        const double dn = (d[0] * fr[0] + d[1] * fr[1]) + d[2] * fr[2];
        for (int k = 0; k < DIM; ++k) d[k] = end ? 0.0 : d[k] - dn * fr[k];
      }
    }
    for (int k = 0; k < 3; ++k) {
      if (a.rates_only) {
        if (a.o_shift) a.o_shift[(int64_t)k * a.n_out + i] = d[k];
      } else {
        a.shift[k][i] = (T)d[k];
      }
    }
  }
  if (a.rates_only) {
    if (a.o_anu)
      for (int k = 0; k < 3; ++k) a.o_anu[(int64_t)k * a.n_out + i] = anu_d[k];
    if (a.o_shift && !a.tvf)   // shift off: zero
      for (int k = 0; k < 3; ++k) a.o_shift[(int64_t)k * a.n_out + i] = 0.0;
    return m_pairs;
  }
  for (int k = 0; k < 3; ++k) a.anu[k][i] = (T)anu_d[k];
  if (TURB) {
    a.ko[i] = (T)k_new;
    a.epso[i] = (T)e_new;
    a.nuto[i] = (T)nut_new;
  }
  // first half density update of the first acoustic sub-step
  const double rho_h = rho_i + a.half_dt * (double)drho_i;
  a.rho[i] = rho_h;
  const T p_h = (T)eos(rho_h, (double)(T)k_new, C.rho0, C.c0, TURB);
  const T v_h = (T)(C.mass / rho_h);
  a.p_out[i] = p_h;
  a.vol_out[i] = v_h;
  write_prec<T, DIM>(a.prec, i, xi, p_h, v_h, Bi);
  return m_pairs;
}

template <typename T, int DIM, int TURB, int L, bool MOM = false>
__global__ __launch_bounds__(256) void k_advection(int n, PairCtx<T> pc, Consts<T> C, AdvArgs<T> a) {
  const int g = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int m = advection_body<T, DIM, TURB, L, MOM>(g / L, g % L, n, pc, C, a);
  count_pairs(pc.pairs, m);
}

// ---------------------------------------------------------------------------
// K8: pressure relaxation.  RKGC pair sum, Eq. (eq-discretize-momentum-p-RKGC),
// with the open-boundary compensation of Eq. (eq-pressure-gradient-obc-B-
// final) (Table 2 variant), velocity kick with the viscous and body force,
// velocity boundary condition of prescribed-velocity buffers, FP64 drift.
// ---------------------------------------------------------------------------
template <typename T>
struct PressArgs {
  const T *p;
  const T* k;               // turbulent kinetic energy (p_eff of the records)
  const double* rho;
  const T* B[6];
  T* v[3];
  const T* anu[3];
  const double* x[3];
  double* xo[3];
  T* xro[3];
  const V4<T>* prec[3];     // pressure records of the neighbours (read)
  V4<T>* drec[2];           // continuity records of the new state (written)
  const T* xrb[3];          // positions at the neighbour-list build (NULL: no list)
  uint32_t* stale_w;        // outgrown-list word of the next positions
  // the radius the list was built with: lrad[1] = 1 for the relative-motion radius
  // (check |x - x_build - u_c t| <= s_i and t <= Δt_ad = lrad[0]), else the
  // cell-size radius (check |x - x_build| <= the skin)
  const double* lrad;
  const float* lskin;
  const T* cell_u[3];
  double t_el;              // time since the build at the end of this sub-step
  const uint32_t* pid;
  const BufDev* bufs;
  const int32_t* bidx;
  uint32_t* flags;
  double dt;
  int64_t step;
  double t;
  int rates_only;
  double* o_ap;
  int64_t n_out;
};

template <typename T, int DIM, int MODE, int L>
__device__ __forceinline__ int pressure_body(int i, int lane, int n, const PairCtx<T>& pc,
                                             const Consts<T>& C, const PressArgs<T>& a) {
  if (i >= n) return 0;
  int m_pairs = 0;
  // the particle's own operands and the head of its list load with its tag
  // (every slot below n holds valid data): none of them waits for the test
  constexpr int NR = DIM == 2 ? (MODE >= 2 ? 2 : 1) : (MODE >= 2 ? 3 : 2);   // record vectors
  const uint32_t ti = pc.tag[i];
  const auto h = list_head<T, DIM, L, NR>(pc, i, lane);
  const T xr_i[3] = {pc.xr[0][i], pc.xr[1][i], pc.xr[2][i]};
  const T xi[3] = {xr_i[0], xr_i[1], DIM == 3 ? xr_i[2] : T(0)};
  const T pi = a.p[i];
  T Bi[6];
  if (MODE >= 2) load_B<T, DIM>(a.B, i, Bi);
  if (!is_real(ti)) {
    if (!a.rates_only && lane == 0) {
      for (int k = 0; k < 3; ++k) {
        a.xo[k][i] = a.x[k][i];
        a.xro[k][i] = xr_i[k];
      }
      const T vw[3] = {T(0), T(0), T(0)};
      write_drec<T, DIM>(a.drec, i, xi, vw, T(0), -pc.vol[i]);
    }
    return m_pairs;
  }
  // operands of the update after the sum: issued before the walk by wide
  // teams (in flight during it), after the sum by narrow ones
  double rho_i = 0.0, xd[3] = {0.0, 0.0, 0.0};
  int qb = -1, c_i = 0;
  T v_i[3] = {T(0), T(0), T(0)}, anu_i[3] = {T(0), T(0), T(0)}, xrb_i[3] = {T(0), T(0), T(0)};
  T vol_i = T(0);
  auto load_update = [&]() {
    rho_i = a.rho[i];
    qb = tag_kind(ti) == kBuffer ? a.bidx[tag_bid(ti)] : -1;
    if (!a.rates_only) {
      for (int k = 0; k < 3; ++k) xd[k] = a.x[k][i];
      for (int k = 0; k < DIM; ++k) {
        v_i[k] = a.v[k][i];
        anu_i[k] = a.anu[k][i];
        if (a.xrb[0]) xrb_i[k] = a.xrb[k][i];
      }
      c_i = pc.cell[i];
      vol_i = pc.vol[i];
    }
  };
  constexpr bool early = hoist_epilogue<L>();
  if (early) load_update();
  // the pair terms in T, their sums in FP64 (a pressure sum cancels to a
  // small fraction of its terms, so T accumulation would add its own
  // rounding of the partial sums to that of the terms)
  double acc[3] = {0.0, 0.0, 0.0}, s[3] = {0.0, 0.0, 0.0};
  for_neighbors_rec<T, DIM, L, NR>(pc, i, lane, xi, a.prec, h,
                                   [&](int j, const T r[3], T r2, const V4<T>* q) {
    ++m_pairs;
    T gW[3];
    if constexpr (f64_kernel<T, DIM>()) {
      double rr;
      const double fd = dw_over_r_d<T>(r, C.inv_h_d, C.kf_d, &rr);
      gW[0] = (T)(fd * (double)r[0]);
      gW[1] = (T)(fd * (double)r[1]);
      gW[2] = T(0);
    } else {
      const T f = dw_over_r<T>(pair_dist(r2), C.inv_h_t, C.kf_t);
      gW[0] = f * r[0];
      gW[1] = f * r[1];
      gW[2] = DIM == 3 ? f * r[2] : T(0);
    }
    const T volw = DIM == 2 ? q[0].d : q[1].a;
    const bool wall = volw < T(0);
    const T Vj = wall ? -volw : volw;
    const T pj_rec = DIM == 2 ? q[0].c : q[0].d;
    if (MODE >= 2) {
      // (p_i B_j + p_j B_i) gradW; wall: p_w = p_i, B_w = B_i
      T Bj[6];
      T pj;
      if (wall) {
        pj = pi;
#pragma unroll
        for (int k = 0; k < 6; ++k) Bj[k] = Bi[k];
      } else {
        pj = pj_rec;
        if (DIM == 2) {
          Bj[0] = q[1].a; Bj[1] = q[1].b; Bj[3] = q[1].c;
          Bj[2] = Bj[4] = Bj[5] = T(0);
        } else {
          Bj[0] = q[1].b; Bj[1] = q[1].c; Bj[2] = q[1].d;
          Bj[3] = q[NR - 1].a; Bj[4] = q[NR - 1].b; Bj[5] = q[NR - 1].c;
        }
      }
      T bj[3], bi[3];
      symv<T, DIM>(Bj, gW, bj);
      symv<T, DIM>(Bi, gW, bi);
      const T vpi = Vj * pi, vpj = Vj * pj;
      acc[0] += (double)(vpi * bj[0] + vpj * bi[0]);
      acc[1] += (double)(vpi * bj[1] + vpj * bi[1]);
      if (DIM == 3) acc[2] += (double)(vpi * bj[2] + vpj * bi[2]);
    } else {
      const T pj = wall ? pi : pj_rec;
      const T w = Vj * (pi + pj);
      acc[0] += (double)(w * gW[0]);
      acc[1] += (double)(w * gW[1]);
      if (DIM == 3) acc[2] += (double)(w * gW[2]);
    }
    s[0] += (double)(Vj * gW[0]);
    s[1] += (double)(Vj * gW[1]);
    if (DIM == 3) s[2] += (double)(Vj * gW[2]);
  });
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    acc[k] = team_sum<L>(acc[k]);
    s[k] = team_sum<L>(s[k]);
  }
  if (lane != 0) return m_pairs;
  if (!early) load_update();
  if (qb >= 0 && a.bufs[qb].p_mode != kPNone) {
    const double pob = a.bufs[qb].p_mode == kPPrescribed
                           ? a.bufs[qb].p_ob * buffer_ramp(a.bufs[qb], a.t)
                           : (double)pi;
    double cc[3];
    if (MODE == 4) {
      const double Bd[6] = {(double)Bi[0], (double)Bi[1], (double)Bi[2],
                            (double)Bi[3], (double)Bi[4], (double)Bi[5]};
      symv<double, DIM>(Bd, s, cc);
    } else {
      cc[0] = s[0]; cc[1] = s[1]; cc[2] = s[2];
    }
    acc[0] -= 2.0 * pob * cc[0];
    acc[1] -= 2.0 * pob * cc[1];
    acc[2] -= 2.0 * pob * cc[2];
  }
  const double inv_rho = 1.0 / rho_i;
  const double ap[3] = {-acc[0] * inv_rho, -acc[1] * inv_rho, -acc[2] * inv_rho};
  if (a.rates_only) {
    for (int k = 0; k < 3; ++k) a.o_ap[(int64_t)k * a.n_out + i] = ap[k];
    return m_pairs;
  }
  double vn[3];
  for (int k = 0; k < 3; ++k)
    vn[k] = (k < DIM) ? (double)v_i[k] + a.dt * (ap[k] + (double)anu_i[k] + C.g[k]) : 0.0;
  if (qb >= 0 && a.bufs[qb].vel_mode == kVelPrescribed) {
    const BufDev& b = a.bufs[qb];
    double y[3];
    to_local(b, xd[0], xd[1], xd[2], y);
    const double u = profile_speed(DIM, b, y, C.seed, a.pid[i], a.step, a.t);
    for (int k = 0; k < DIM; ++k) vn[k] = u * b.frame[k];
  }
  const int c = c_i;
  const int cc3[3] = {c % pc.nx, (c / pc.nx) % pc.ny, c / (pc.nx * pc.ny)};
  bool bad = false;
  T xnew[3], vnew[3] = {T(0), T(0), T(0)};
  double d2 = 0.0;   // displacement since the neighbour-list build
  for (int k = 0; k < 3; ++k) {
    if (k < DIM) {
      const T vt = (T)vn[k];
      a.v[k][i] = vt;
      const double xn = xd[k] + a.dt * (double)vt;
      a.xo[k][i] = xn;
      const double rel = xn - cell_centre(C.grid.lo[k], cc3[k], C.grid.cs);
      if (!(fabs(rel) <= 0.5 * C.grid.cs + C.skin)) bad = true;
      if (a.xrb[0]) {
        const double dd = rel - (double)xrb_i[k];
        d2 += dd * dd;
      }
      a.xro[k][i] = (T)rel;
      xnew[k] = (T)rel;
      vnew[k] = vt;
    } else {
      a.xo[k][i] = xd[k];
      a.xro[k][i] = xr_i[k];
      xnew[k] = xr_i[k];
    }
  }
  if (a.xrb[0] && a.lrad[1] > 0.0) {
    // relative-motion radius: the displacement less the cell's drift
    d2 = 0.0;
    for (int k = 0; k < DIM; ++k) {
      const double dd = ((double)xnew[k] - (double)xrb_i[k]) - (double)a.cell_u[k][c] * a.t_el;
      d2 += dd * dd;
    }
    const double s = (double)a.lskin[i];
    if (!(d2 <= s * s) || !(a.t_el <= a.lrad[0] * (1.0 + 1e-9))) atomicOr(a.stale_w, 1u);
  } else if (a.xrb[0] && !(d2 <= C.skin * C.skin)) {
    atomicOr(a.stale_w, 1u);
  }
  T plo = T(0);   // the FP64 remainder of p_i (2D FP32: continuity pressure differences)
  if constexpr (f64_kernel<T, DIM>())
    plo = (T)(eos(rho_i, C.turbulence ? (double)a.k[i] : 0.0, C.rho0, C.c0, C.turbulence) -
              (double)pi);
  write_drec<T, DIM>(a.drec, i, xnew, vnew, pi, vol_i, plo);
  if (bad) atomicOr(a.flags, kFlagSkin);
  return m_pairs;
}

template <typename T, int DIM, int MODE, int L>
__global__ __launch_bounds__(256) void k_pressure(int n, PairCtx<T> pc, Consts<T> C, PressArgs<T> a) {
  const int g = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  // an outgrown list stays outgrown for the rest of the step
  if (g == 0 && a.stale_w && pc.stale && *pc.stale) atomicOr(a.stale_w, 1u);
  const int m = pressure_body<T, DIM, MODE, L>(g / L, g % L, n, pc, C, a);
  count_pairs(pc.pairs, m);
}

// ---------------------------------------------------------------------------
// K9: density relaxation.  Continuity with the Riemann intermediate velocity,
// Eqs. (discretize-continuity-equ-riemann) and (eq-intermediate-vel):
// (v_i - v*) . gradW_ij = v_ij . gradW_ij / 2 + (p_i - p_j) / (2 rho0 c0) W'
// with the Riemann axis from i to j; walls: v_w = 0, p_w = p_i.  Second half
// density update (FP64) and, if another sub-step follows, its first half
// update, pressure and volume.
// ---------------------------------------------------------------------------
template <typename T>
struct DensArgs {
  const T* v[3];
  const T* p;
  double* rho;
  T* drho;
  const T* k;
  T *p_out, *vol_out;
  double half_dt;
  int last;
  int rates_only;
  double* o_drho;
  const V4<T>* drec[2];   // continuity records of the neighbours (read)
  V4<T>* prec[3];         // pressure records of the next sub-step (written)
  const T* B[6];
};

template <typename T, int DIM, int TURB, int L>
__global__ __launch_bounds__(256) void k_density(int n, PairCtx<T> pc, Consts<T> C,
                                                 DensArgs<T> a) {
  const int g = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int i = g / L, lane = g % L;
  long long cnt = 0;
  if (i < n) {
    // the tag, the position and the head of the list load together
    const uint32_t ti = pc.tag[i];
    const auto h = list_head<T, DIM, L, 2>(pc, i, lane);
    const T xi[3] = {pc.xr[0][i], pc.xr[1][i], DIM == 3 ? pc.xr[2][i] : T(0)};
    if (is_real(ti)) {
      const T vi[3] = {a.v[0][i], a.v[1][i], DIM == 3 ? a.v[2][i] : T(0)};
      const T pi = a.p[i];
      // operands of the update after the sum: issued before the walk by
      // wide teams, after the sum by narrow ones
      const bool next = !a.rates_only && !a.last;
      double rho_i = 0.0, k_i = 0.0;
      // 2D FP32: p_i in FP64 from the density it came from (Eq. eos), so
      // that p_i - p_j keeps its digits with the record's p + p_lo
      double pid = 0.0;
      if constexpr (f64_kernel<T, DIM>())
        pid = eos(a.rho[i], C.turbulence ? (double)a.k[i] : 0.0, C.rho0, C.c0, C.turbulence);
      T Bw[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
      auto load_update = [&]() {
        rho_i = a.rho[i];
        if (next) load_B<T, DIM>(a.B, i, Bw);
        if (TURB && next) k_i = (double)a.k[i];
      };
      constexpr bool early = hoist_epilogue<L>();
      if (early) load_update();
      double sum = 0.0;   // FP64 sum of T terms (near-cancelling, see the pressure pass)
      int m = 0;
      for_neighbors_rec<T, DIM, L, 2>(pc, i, lane, xi, a.drec, h,
                                      [&](int j, const T r[3], T r2, const V4<T>* q) {
        const T rr = pair_dist(r2);
        const T f = dw_over_r<T>(rr, C.inv_h_t, C.kf_t);
        const T volw = DIM == 2 ? q[1].b : q[1].d;
        const bool wall = volw < T(0);
        const T Vj = wall ? -volw : volw;
        T vr, dp;
        if (wall) {
          vr = vi[0] * r[0] + vi[1] * r[1] + vi[2] * r[2];
          dp = T(0);
        } else {
          const T vj0 = DIM == 2 ? q[0].c : q[0].d;
          const T vj1 = DIM == 2 ? q[0].d : q[1].a;
          const T vj2 = DIM == 2 ? T(0) : q[1].b;
          const T pj = DIM == 2 ? q[1].a : q[1].c;
          vr = (vi[0] - vj0) * r[0] + (vi[1] - vj1) * r[1] +
               (DIM == 3 ? (vi[2] - vj2) * r[2] : T(0));
          if constexpr (f64_kernel<T, DIM>())
            dp = (T)(pid - ((double)pj + (double)q[1].c));
          else
            dp = pi - pj;
        }
        sum += (double)(Vj * f * (T(0.5) * vr + dp * C.inv_2rc0_t * rr));
        ++m;
      });
      cnt = m;
      sum = team_sum<L>(sum);
      if (lane == 0) {
        if (!early) load_update();
        const double drho = 2.0 * rho_i * sum;
        if (a.rates_only) {
          a.o_drho[i] = drho;
        } else {
          a.drho[i] = (T)drho;
          double rho_n = rho_i + a.half_dt * drho;
          if (!a.last) {
            rho_n = rho_n + a.half_dt * drho;
            const T p_n = (T)eos(rho_n, k_i, C.rho0, C.c0, TURB);
            const T v_n = (T)(C.mass / rho_n);
            a.p_out[i] = p_n;
            a.vol_out[i] = v_n;
            write_prec<T, DIM>(a.prec, i, xi, p_n, v_n, Bw);
          }
          a.rho[i] = rho_n;
        }
      }
    } else if (!a.rates_only && !a.last && lane == 0) {
      a.p_out[i] = T(0);
      a.vol_out[i] = (T)C.Vw;
      const T Iw[6] = {T(1), T(0), T(0), T(1), T(0), T(1)};
      write_prec<T, DIM>(a.prec, i, xi, T(0), -(T)C.Vw, Iw);
    }
  }
  count_pairs(pc.pairs, cnt);
}

template <typename T>
struct PvArgs {
  const double* rho;
  const T* k;
  const uint32_t* tag;
  T *p, *vol;
  double* o_p;
  const T* xr[3];
  const T* v[3];
  const T* B[6];
  V4<T>* prec[3];
  V4<T>* drec[2];
};

// p and V from the current density, and the j-side records of the pressure
// and continuity passes at the current state (rates at a state).
template <typename T, int DIM>
__global__ void k_prepare_pv(int n, Consts<T> C, PvArgs<T> a) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T x[3] = {a.xr[0][i], a.xr[1][i], DIM == 3 ? a.xr[2][i] : T(0)};
  if (!is_real(a.tag[i])) {
    a.p[i] = T(0);
    a.vol[i] = (T)C.Vw;
    if (a.o_p) a.o_p[i] = 0.0;
    const T Iw[6] = {T(1), T(0), T(0), T(1), T(0), T(1)};
    const T vw[3] = {T(0), T(0), T(0)};
    write_prec<T, DIM>(a.prec, i, x, T(0), -(T)C.Vw, Iw);
    write_drec<T, DIM>(a.drec, i, x, vw, T(0), -(T)C.Vw);
    return;
  }
  const double r = a.rho[i];
  const double pp = eos(r, C.turbulence ? (double)a.k[i] : 0.0, C.rho0, C.c0, C.turbulence);
  const T pt = (T)pp, vt = (T)(C.mass / r);
  a.p[i] = pt;
  a.vol[i] = vt;
  if (a.o_p) a.o_p[i] = pp;
  T B[6];
  load_B<T, DIM>(a.B, i, B);
  const T v[3] = {a.v[0][i], a.v[1][i], DIM == 3 ? a.v[2][i] : T(0)};
  write_prec<T, DIM>(a.prec, i, x, pt, vt, B);
  write_drec<T, DIM>(a.drec, i, x, v, pt, vt, f64_kernel<T, DIM>() ? (T)(pp - (double)pt) : T(0));
}

// ---------------------------------------------------------------------------
// K11: max |v|^2, max nu_t over real particles and a non-finite flag.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_reduce_part(int n, const int32_t* n_extra, int n_max,
                                                     const T* v0, const T* v1,
                                                     const T* v2, const double* rho,
                                                     const T* nut, const uint32_t* tag,
                                                     int turb, double* part) {
  __shared__ double sm[2][256 / kWave];
  // slots: n, plus the particles the buffer update just appended
  if (n_extra) n = min(n + *n_extra, n_max);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double a = 0.0, b = 0.0;
  if (i < n && is_real(tag[i])) {
    const double x = v0[i], y = v1[i], z = v2[i];
    a = (x * x + y * y) + z * z;
    const double r = rho[i];
    if (!(a == a) || !(r == r) || isinf(a) || isinf(r)) a = INFINITY;
    if (turb) b = nut[i];
  }
  a = wave_max(a);
  b = wave_max(b);
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  if (lane == 0) { sm[0][wid] = a; sm[1][wid] = b; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x / kWave); ++w) {
      a = fmax(a, sm[0][w]);
      b = fmax(b, sm[1][w]);
    }
    part[2 * blockIdx.x] = sm[0][0] > a ? sm[0][0] : a;
    part[2 * blockIdx.x + 1] = sm[1][0] > b ? sm[1][0] : b;
  }
}

// K11 after a buffer update, in one launch: max |v|^2 and max nu_t of the
// updated state, one pair per workgroup (the host takes the maxima of the
// pairs: exact and order-independent), the per-buffer counts, the error
// flags and the next particle id, all written straight into the pinned host
// buffer `rb` (its device address) in the counters' layout -- counts in
// [0, 1032), flags and id in [1032, 1035), the pairs after word 1040 -- so
// that the update needs no copy.  Plain stores: no two workgroups write one
// word.
// Cell keys of the updated arrays for a build launched after the
// reduction (key == NULL: none).
struct KeyOut {
  const double* x[3];
  GridDev g;
  int32_t *key, *slot, *count;
};

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_reduce_post(int n, int n_max, int32_t* counters,
                                                     const T* v0, const T* v1, const T* v2,
                                                     const double* rho, const T* nut,
                                                     const uint32_t* tag, int turb,
                                                     uint32_t* flags,
                                                     const uint64_t* next_pid, int n_alive,
                                                     int32_t* __restrict__ ns,
                                                     int32_t* __restrict__ rb, KeyOut ko,
                                                     const uint32_t* __restrict__ stale) {
  __shared__ double sm[2][256 / kWave];
  if (blockIdx.x == 0)
    for (int k = threadIdx.x; k < 1032; k += blockDim.x) rb[k] = counters[k];
  if (blockIdx.x == 0 && threadIdx.x < kWave) {
    // sizes of the next cell build, for a build launched before the host
    // has read the counts: {n_in, n_out, skip (the injection failed)}
    long long del = 0;
    for (int b = threadIdx.x; b < 256; b += kWave) del += counters[512 + b];
    del = wave_sum_ll(del);
    if (threadIdx.x == 0) {
      const bool cap = (*flags & kFlagCapacity) != 0;
      const int inj = cap ? 0 : counters[1024];
      ns[0] = n + inj;
      ns[1] = n_alive + inj - (int)del;
      ns[2] = cap ? 1 : 0;
    }
  }
  n = min(n + counters[1024], n_max);
  // the next build's keys, unless the injection failed (its kernels are
  // skipped then, and the counts must stay clear)
  const bool keys = ko.key && (*flags & kFlagCapacity) == 0;
  double a = 0.0, b = 0.0;
  // a block-uniform trip count: every lane of a wavefront takes part in the
  // run-aggregated slot atomics of cell_key_slot
  for (int i0 = blockIdx.x * blockDim.x; i0 < n; i0 += gridDim.x * blockDim.x) {
    const int i = i0 + (int)threadIdx.x;
    if (keys)
      cell_key_slot<DIM>(i, n, ko.x[0], ko.x[1], ko.x[2], tag, ko.g, ko.key, ko.slot, ko.count,
                         flags);
    if (i >= n || !is_real(tag[i])) continue;
    const double x = v0[i], y = v1[i], z = v2[i];
    double q = (x * x + y * y) + z * z;
    const double r = rho[i];
    if (!(q == q) || !(r == r) || isinf(q) || isinf(r)) q = INFINITY;
    a = fmax(a, q);
    if (turb && (double)nut[i] > b) b = (double)nut[i];   // never -0.0
  }
  a = wave_max(a);
  b = wave_max(b);
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  if (lane == 0) { sm[0][wid] = a; sm[1][wid] = b; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) {
      a = fmax(a, sm[0][w]);
      b = fmax(b, sm[1][w]);
    }
    double* part = reinterpret_cast<double*>(rb + 1040) + 2 * blockIdx.x;
    part[0] = a;
    part[1] = b;
    if (blockIdx.x == 0) {
      rb[1032] = (int32_t)*flags;
      rb[1035] = (int32_t)(stale[0] | stale[1]);   // the step's list outgrown
      const uint64_t np = *next_pid;
      rb[1033] = (int32_t)(uint32_t)(np & 0xFFFFFFFFull);
      rb[1034] = (int32_t)(uint32_t)(np >> 32);
    }
  }
}

// The coming advection step's Δt_ad from per-workgroup maxima {|v|^2,
// nu_t} (the post-update reduction's, in the read-back buffer, or a fresh
// reduction's), formed as the host forms it (dual criteria, Sec. 2.3), for
// the list radius of a build.  lrad[0] = Δt_ad, 0 when not finite.  One
// workgroup of 1024 lanes: the read-back buffer's (at most 1024) pairs sit
// in host memory, and one load per lane keeps them all in flight at once.
constexpr int kListDtThreads = 1024;
__global__ __launch_bounds__(kListDtThreads) void k_list_dt(int nb, const double* __restrict__ part,
                                                            double h, double cfl, double u_ref,
                                                            double nu_l, double* lrad) {
  double a = 0.0, b = 0.0;
  for (int q = threadIdx.x; q < nb; q += blockDim.x) {
    a = fmax(a, part[2 * q]);
    b = fmax(b, part[2 * q + 1]);
  }
  a = wave_max(a);
  b = wave_max(b);
  __shared__ double sm[2][kListDtThreads / kWave];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  if (lane == 0) {
    sm[0][wid] = a;
    sm[1][wid] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) {
      a = fmax(a, sm[0][w]);
      b = fmax(b, sm[1][w]);
    }
    const double dt = cfl * fmin(h / fmax(sqrt(a), u_ref), h * h / (2.0 * (nu_l + b)));
    lrad[0] = (dt > 0.0 && dt < INFINITY) ? dt : 0.0;
  }
}

// Per cell of a fresh build, for the relative-motion list radius: u_c, the
// mean velocity of the cell's moving (real) particles, and for each of its
// particles s_i = kListSkinFactor |v_i - u_c| Δt_ad + kListSkinFloor h, the
// deviation from drifting with u_c allowed over the step (a wall, which
// does not move, deviates by |u_c| Δt_ad).  Skipped when Δt_ad is unknown.
#ifndef SPHX_LIST_SKIN_FACTOR
#define SPHX_LIST_SKIN_FACTOR 2.0
#endif
#ifndef SPHX_LIST_SKIN_FLOOR
#define SPHX_LIST_SKIN_FLOOR 0.05
#endif
constexpr double kListSkinFactor = SPHX_LIST_SKIN_FACTOR;
constexpr double kListSkinFloor = SPHX_LIST_SKIN_FLOOR;

// A team of skin_lanes<DIM>() lanes per cell (3D cells hold ~40 particles,
// 2D ~10): coalesced loads of the cell's members and a butterfly sum
// (measured on the 3.75M-particle mixer: one thread per cell walking its
// members took 285 us).
template <int DIM>
constexpr int skin_lanes() {
  return DIM == 3 ? 64 : 16;
}

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_cell_skin(int ncell, const int32_t* __restrict__ cs,
                                                   const T* v0, const T* v1, const T* v2,
                                                   const uint32_t* __restrict__ tag,
                                                   const double* __restrict__ lrad, double h,
                                                   const int32_t* __restrict__ ns, T* u0, T* u1,
                                                   T* u2, float* skin) {
  constexpr int CL = skin_lanes<DIM>();
  if (ns && ns[2]) return;
  const double dt = lrad[0];
  if (!(dt > 0.0)) return;
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = g / CL, lane = g % CL;
  const bool valid = c < ncell;
  int j0 = 0, j1 = 0;
  if (valid) {
    j0 = cs[c];
    j1 = cs[c + 1];
  }
  double su[3] = {0.0, 0.0, 0.0}, m = 0.0;
  for (int j = j0 + lane; j < j1; j += CL) {
    if (!is_real(tag[j])) continue;
    su[0] += (double)v0[j];
    su[1] += (double)v1[j];
    if (DIM == 3) su[2] += (double)v2[j];
    m += 1.0;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) su[k] = team_sum<CL>(su[k]);
  m = team_sum<CL>(m);
  if (!valid) return;
  const double inv = m > 0.0 ? 1.0 / m : 0.0;
  const T u[3] = {(T)(su[0] * inv), (T)(su[1] * inv), (T)(su[2] * inv)};
  if (lane == 0) {
    u0[c] = u[0];
    u1[c] = u[1];
    if (DIM == 3) u2[c] = u[2];
  }
  // a wall does not move: from drifting with u_c it deviates by |u_c| t, and
  // s_wall + |u_c(i) - u_c| dt_ad >= |u_c(i)| dt_ad bounds its pairs
  const double s_wall = sqrt(su[0] * su[0] + su[1] * su[1] + su[2] * su[2]) * inv * dt;
  for (int j = j0 + lane; j < j1; j += CL) {
    double sj = s_wall;
    if (is_real(tag[j])) {
      const double d0 = (double)v0[j] - (double)u[0], d1 = (double)v1[j] - (double)u[1];
      const double d2 = DIM == 3 ? (double)v2[j] - (double)u[2] : 0.0;
      sj = kListSkinFactor * sqrt(d0 * d0 + d1 * d1 + d2 * d2) * dt + kListSkinFloor * h;
    }
    skin[j] = (float)sj;
  }
}

__global__ __launch_bounds__(256) void k_reduce_final(int nb, const double* part, double* out,
                                                      const uint32_t* flags) {
  double a = 0.0, b = 0.0;
  for (int q = threadIdx.x; q < nb; q += blockDim.x) {
    a = fmax(a, part[2 * q]);
    b = fmax(b, part[2 * q + 1]);
  }
  __shared__ double sm[2][256 / kWave];
  a = wave_max(a);
  b = wave_max(b);
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  if (lane == 0) { sm[0][wid] = a; sm[1][wid] = b; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) {
      a = fmax(a, sm[0][w]);
      b = fmax(b, sm[1][w]);
    }
    out[0] = a;
    out[1] = b;
    // the error flags travel with the maxima (one read-back per step)
    reinterpret_cast<uint32_t*>(out + 2)[0] = *flags;
  }
}

// ---------------------------------------------------------------------------
// K4: neighbour lists with the FP64 predicate (parity / diagnostics).
// ---------------------------------------------------------------------------
template <int DIM, int FILL>
__global__ void k_neighbors(int n, const double* x0, const double* x1, const double* x2,
                            const int32_t* cell, const int32_t* cstart, int nx, int ny,
                            double rc2, int32_t* row, int32_t* col, int64_t cap) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = cell[i];
  const int cx = c % nx, cy = (c / nx) % ny, cz = c / (nx * ny);
  const double xi0 = x0[i], xi1 = x1[i], xi2 = x2[i];
  int m = 0;
  int64_t o = FILL ? row[i] : 0;
  constexpr int zr = DIM == 3 ? 1 : 0;
  for (int dz = -zr; dz <= zr; ++dz)
    for (int dy = -1; dy <= 1; ++dy) {
      const int base = ((cz + dz) * ny + (cy + dy)) * nx + cx;
      for (int j = cstart[base - 1]; j < cstart[base + 2]; ++j) {
        if (j == i) continue;
        const double d0 = __dsub_rn(xi0, x0[j]), d1 = __dsub_rn(xi1, x1[j]),
                     d2 = __dsub_rn(xi2, x2[j]);
        const double r2 = __dadd_rn(__dadd_rn(__dmul_rn(d0, d0), __dmul_rn(d1, d1)),
                                    __dmul_rn(d2, d2));
        if (r2 < rc2) {
          if (FILL && o + m < cap) col[o + m] = j;
          ++m;
        }
      }
    }
  if (!FILL) row[i] = m;
}

// The pairs the pair passes of a step visit: particle i's candidates (the
// per-step list, or the cell stencil when the list is off) that pass the
// passes' own test |r_ij|^2 < (2h)^2 on cell-relative positions in the pair
// precision, in visiting order; none for particles that are not real.
template <typename T, int DIM, int FILL>
__global__ void k_walk_pairs(int n, PairCtx<T> pc, int32_t* row, int32_t* col, int64_t cap) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int m = 0;
  const int64_t o = FILL ? row[i] : 0;
  if (is_real(pc.tag[i])) {
    const T xi[3] = {pc.xr[0][i], pc.xr[1][i], DIM == 3 ? pc.xr[2][i] : T(0)};
    for_neighbors<T, DIM, 1>(pc, i, 0, xi, [&](int j, const T*, T) {
      if (FILL && o + m < cap) col[o + m] = j;
      ++m;
    });
  }
  if (!FILL) row[i] = m;
}

template <typename T, int DIM>
__global__ void k_export_B(int n, const T* B0, const T* B1, const T* B2, const T* B3,
                           const T* B4, const T* B5, double* out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double b[6] = {(double)B0[i], (double)B1[i], DIM == 3 ? (double)B2[i] : 0.0,
                 (double)B3[i], DIM == 3 ? (double)B4[i] : 0.0,
                 DIM == 3 ? (double)B5[i] : 0.0};
  const int64_t N = n;
  out[0 * N + i] = b[0];
  out[1 * N + i] = b[1];
  out[2 * N + i] = b[2];
  out[3 * N + i] = b[1];
  out[4 * N + i] = b[3];
  out[5 * N + i] = b[4];
  out[6 * N + i] = b[2];
  out[7 * N + i] = b[4];
  out[8 * N + i] = b[5];
}

// End of the advection step with the transport-velocity shift: real
// particles advance by the shift summed on the start-of-step state (zero for
// prescribed-velocity buffers), FP64 master position and cell-relative copy.
// No neighbour is read, so the update is in place.
template <typename T, int DIM>
__global__ void k_shift_apply(int n, const uint32_t* __restrict__ tag, const T* s0, const T* s1,
                              const T* s2, double* x0, double* x1, double* x2, T* r0, T* r1,
                              T* r2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || tag_kind(tag[i]) > kBuffer) return;
  const T d[3] = {s0[i], s1[i], DIM == 3 ? s2[i] : T(0)};
  x0[i] += (double)d[0];
  x1[i] += (double)d[1];
  r0[i] += d[0];
  r1[i] += d[1];
  if (DIM == 3) {
    x2[i] += (double)d[2];
    r2[i] += d[2];
  }
}

// ---------------------------------------------------------------------------
// host-side argument assembly
// ---------------------------------------------------------------------------
inline int nblk(int64_t n) { return (int)((n + 255) / 256) + (n == 0); }

// Lanes per particle of the neighbour passes: enough wavefronts to hide the
// latency of the candidate loads on 256 CUs at small particle counts, one
// lane per particle once the grid alone fills the machine (measured on
// MI355X, 2D: at 57k particles L = 4 is fastest, 0.55x the step time of
// L = 1; at 640k and 2.56M particles L = 1 is fastest).
// Lanes per particle (measured on 2D workloads): enough wavefronts to cover
// the load latency at small sizes, one lane per particle once the chip is
// full.  The correction's stencil scan walks ~3x the candidates of the list
// passes and takes twice the lanes (two at most sizes: 160 against 242 us at
// 640k particles, 590 against 731 us at 2.56M).  In 3D (3.75M particles) the
// passes take 2 lanes (pressure 2.7 against 3.3 ms with one) and the
// correction 4 (6.9 against 7.6 ms with two).  With the relative-motion
// list radius (~100 entries) FP64 3D passes take four lanes at every size
// (the mixer: 26.5 against 29.3 ms per step with two), FP32 keeps two (15.1
// against 15.7 with four, 19.3 with one).
inline int team_lanes(const sph_ctx* c) {
  if (c->team_override > 0) return c->team_override;
  const int64_t n = c->n_total;
  if (c->P.dim == 3)   // ~100-170 list entries per particle: more lanes at every size
    return (n <= 1000000 || c->P.precision == SPH_FP64) ? 4 : 2;
  if (n <= 100000) return 4;
  if (n <= 450000) return 2;
  return 1;
}

inline int corr_lanes(const sph_ctx* c, int64_t n) {
  if (c->corr_override > 0) return c->corr_override;
  if (c->team_override > 0) return c->team_override;
  if (c->P.dim == 3) return n <= 100000 ? 8 : 4;   // ~1000 stencil candidates
  if (n <= 100000) return 8;
  if (n <= 260000) return 4;
  return 2;
}

#define SPHX_TEAM_SWITCH(L, ...)                                   \
  switch (L) {                                                     \
    case 1: { constexpr int TL = 1; __VA_ARGS__; } break;          \
    case 2: { constexpr int TL = 2; __VA_ARGS__; } break;          \
    case 4: { constexpr int TL = 4; __VA_ARGS__; } break;          \
    default: { constexpr int TL = 8; __VA_ARGS__; } break;         \
  }

// The 3D moment over the list just written: B of every particle (the
// correction's second kernel).  ns / n: the sizes as for the list.
template <typename T, int DIM>
hipError_t moment_impl(sph_ctx* c, const int32_t* ns, int64_t n) {
  if constexpr (DIM == 3) {
    Consts<T> C = make_consts<T>(c);
    PairCtx<T> pl = make_pc<T>(c, c->F.xr, c->F.x[0].cur);
    pl.nbr = c->F.nbr;
    pl.ncnt = c->F.ncnt;
    pl.stale = nullptr;
    CorrArgs<T> am;
    for (int k = 0; k < 3; ++k) am.x[k] = c->F.x[k].live();
    am.bufs = c->S.bufs;
    for (int k = 0; k < 6; ++k) am.B[k] = tp<T>(c->F.B[k]);
    am.flags = c->S.flags;
    am.mirror = c->P.obc_mode >= 3 ? 1 : 0;
    for (int k = 0; k < 2; ++k) am.arec[k] = tp<V4<T>>(c->F.arec[k]);
    NbrOut<T> nb{};
    const int Lm = team_lanes(c);
    SPHX_TEAM_SWITCH(Lm, launch_pass(c, &k_correction<T, DIM, TL, false, true, true>, nblk(n * TL), (int)n, pl, C, am, nb, ns));
    c->B_pending = false;
  }
  return hipGetLastError();
}

template <typename T, int DIM>
hipError_t correction_impl(sph_ctx* c, const int32_t* ns, int64_t n_grid, bool tight,
                           bool moment) {
  Consts<T> C = make_consts<T>(c);
  c->nbr_valid = false;
  tight = tight && c->use_nbr;
  if (tight) {
    const int nc = c->grid.ncell;
    k_cell_skin<T, DIM><<<(int)(((int64_t)nc * skin_lanes<DIM>() + 255) / 256), 256, 0, c->stream>>>(
        nc, c->S.cell_start, tp<T>(c->F.v[0].live()), tp<T>(c->F.v[1].live()),
        tp<T>(c->F.v[2].live()), c->F.tag.live(), c->S.lrad, c->P.h, ns, tp<T>(c->F.cell_u[0]),
        tp<T>(c->F.cell_u[1]), tp<T>(c->F.cell_u[2]), c->F.lskin);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  PairCtx<T> pc = make_pc<T>(c, c->F.xr, c->F.x[0].cur);   // stencil: no list yet
  CorrArgs<T> a;
  for (int k = 0; k < 3; ++k) a.x[k] = c->F.x[k].live();
  a.bufs = c->S.bufs;
  for (int k = 0; k < 6; ++k) a.B[k] = tp<T>(c->F.B[k]);
  a.flags = c->S.flags;
  a.mirror = c->P.obc_mode >= 3 ? 1 : 0;
  a.arec[0] = a.arec[1] = nullptr;
  NbrOut<T> nb;
  nb.nbr = c->F.nbr;
  nb.ncnt = c->F.ncnt;
  nb.stride = c->cap;
  nb.K = c->F.nbr_k;
  for (int k = 0; k < 3; ++k) nb.xb[k] = tp<T>(c->F.xrb[k]);
  nb.flags = c->S.flags;
  nb.stale = c->S.stale;
  const double rl = c->P.cell_size * (1.0 + 2e-6);
  nb.rl2 = (T)(rl * rl);
  nb.stage = nullptr;
  nb.kstage = 0;
  nb.queue = nullptr;
  nb.tight = tight ? 1 : 0;
  nb.lrad = c->S.lrad;
  nb.lskin = c->F.lskin;
  for (int k = 0; k < 3; ++k) nb.xs[k] = c->F.xr32[k];
  for (int k = 0; k < 3; ++k) nb.cell_u[k] = tp<T>(c->F.cell_u[k]);
  nb.two_h = (T)(2.0 * c->P.h);
  nb.rl = (T)rl;
  nb.cell_q = c->S.cell_q;
  nb.q_rl = (T)(rl * (1.0 + 1e-5));
  nb.q_w = (T)(4.0 / c->P.cell_size);
  const int64_t n = ns ? n_grid : c->n_total;
  const int L = corr_lanes(c, c->n_total);
  if (c->use_nbr && split_correction<DIM>()) {
    // the list, then the moment over it (its own lane count, the passes');
    // under profiling the section's events bracket both kernels
    hipEvent_t pa = c->prof.ext_a, pb = c->prof.ext_b;
    c->prof.ext_a = c->prof.ext_b = nullptr;
    if (pa) (void)hipEventRecord(pa, c->stream);
    SPHX_TEAM_SWITCH(L, launch_pass(c, &k_correction<T, DIM, TL, true, false>, nblk(n * TL), (int)n, pc, C, a, nb, ns));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // B now, or in the step's advection pass (laminar: it walks the same
    // list); until then B of this state is pending
    if (moment || c->P.turbulence) {
      e = moment_impl<T, DIM>(c, ns, n);
      if (e != hipSuccess) return e;
    } else {
      c->B_pending = true;
    }
    if (pb) (void)hipEventRecord(pb, c->stream);
  } else if (c->use_nbr) {
    SPHX_TEAM_SWITCH(L, launch_pass(c, &k_correction<T, DIM, TL, true>, nblk(n * TL), (int)n, pc, C, a, nb, ns));
  } else {
    SPHX_TEAM_SWITCH(L, launch_pass(c, &k_correction<T, DIM, TL, false>, nblk(n * TL), (int)n, pc, C, a, nb, ns));
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && c->use_nbr) c->nbr_valid = true;
  return e;
}

// The 3D laminar list passes form B in the advection pass (advection_body,
// MOM), from the same list walk; the correction then only writes the list
// when the step follows at once (sph_advance).
bool advection_forms_B(const sph_ctx* c, bool rates_only) {
  return c->P.dim == 3 && !c->P.turbulence && !rates_only && c->use_nbr && c->nbr_valid;
}

template <typename T, int DIM>
hipError_t advection_impl(sph_ctx* c, double dt_adv, double dt_sub, bool rates_only,
                          const sph_rates* out) {
  Consts<T> C = make_consts<T>(c);
  PairCtx<T> pc = make_pc<T>(c, c->F.xr, c->F.x[0].cur);
  AdvArgs<T> a;
  Fields& F = c->F;
  for (int k = 0; k < 3; ++k) {
    a.v[k] = tp<T>(F.v[k].live());
    a.anu[k] = tp<T>(F.anu[k]);
  }
  a.rho = F.rho.live();
  a.drho = tp<T>(F.drho.live());
  for (int k = 0; k < 6; ++k) a.B[k] = tp<T>(F.B[k]);
  a.k = tp<T>(F.k.live());
  a.eps = tp<T>(F.eps.live());
  a.nut = tp<T>(F.nut.live());
  a.ko = tp<T>(F.k.other());
  a.epso = tp<T>(F.eps.other());
  a.nuto = tp<T>(F.nut.other());
  a.p_out = tp<T>(F.p.other());
  a.vol_out = tp<T>(F.vol.other());
  a.bufs = c->S.bufs;
  a.bidx = c->S.bidx;
  a.dt_adv = dt_adv;
  a.half_dt = 0.5 * dt_sub;
  a.rates_only = rates_only ? 1 : 0;
  a.o_anu = out ? out->anu : nullptr;
  if (rates_only) pc.pairs = nullptr;
  a.o_gradv = out ? out->gradv : nullptr;
  a.o_dk = out ? out->dk : nullptr;
  a.o_deps = out ? out->deps : nullptr;
  a.n_out = c->n_total;
  for (int k = 0; k < 3; ++k) a.prec[k] = tp<V4<T>>(F.prec[k]);
  for (int k = 0; k < 3; ++k) a.arec[k] = tp<V4<T>>(F.arec[k]);
  a.tvf = F.shift[0] && (!rates_only || (out && out->shift)) ? 1 : 0;
  a.tvf_c = -2.0 * c->P.tvf_alpha * c->P.h * c->P.h;
  a.two_h = 2.0 * c->P.h;
  for (int k = 0; k < 3; ++k) a.x[k] = F.x[k].live();
  for (int k = 0; k < 3; ++k) a.shift[k] = tp<T>(F.shift[k]);
  a.o_shift = out ? out->shift : nullptr;
  for (int k = 0; k < 3; ++k) a.cor.x[k] = F.x[k].live();
  a.cor.bufs = c->S.bufs;
  for (int k = 0; k < 6; ++k) a.cor.B[k] = tp<T>(F.B[k]);
  a.cor.flags = c->S.flags;
  a.cor.mirror = c->P.obc_mode >= 3 ? 1 : 0;
  a.cor.arec[0] = a.cor.arec[1] = nullptr;
  const int64_t n = c->n_total;
  const int L = team_lanes(c);
  if (c->P.turbulence) {
    SPHX_TEAM_SWITCH(L, launch_pass(c, &k_advection<T, DIM, 1, TL>, nblk(n * TL), (int)n, pc, C, a));
  } else if (advection_forms_B(c, rates_only)) {
    if constexpr (DIM == 3)
      SPHX_TEAM_SWITCH(L, launch_pass(c, &k_advection<T, DIM, 0, TL, true>, nblk(n * TL), (int)n, pc, C, a));
  } else {
    SPHX_TEAM_SWITCH(L, launch_pass(c, &k_advection<T, DIM, 0, TL>, nblk(n * TL), (int)n, pc, C, a));
  }
  if (advection_forms_B(c, rates_only)) c->B_pending = false;
  return hipGetLastError();
}

template <typename T, int DIM>
hipError_t pressure_impl(sph_ctx* c, double dt, bool rates_only, const sph_rates* out) {
  Consts<T> C = make_consts<T>(c);
  PairCtx<T> pc = make_pc<T>(c, c->F.xr, c->F.x[0].cur);
  Fields& F = c->F;
  PressArgs<T> a;
  a.p = tp<T>(F.p.live());
  a.k = tp<T>(F.k.live());
  a.rho = F.rho.live();
  for (int k = 0; k < 6; ++k) a.B[k] = tp<T>(F.B[k]);
  for (int k = 0; k < 3; ++k) {
    a.v[k] = tp<T>(F.v[k].live());
    a.anu[k] = tp<T>(F.anu[k]);
    a.x[k] = F.x[k].live();
    a.xo[k] = F.x[k].other();
    a.xro[k] = tp<T>(F.xr[k].other());
    a.xrb[k] = pc.nbr ? tp<T>(F.xrb[k]) : nullptr;
    a.prec[k] = tp<V4<T>>(F.prec[k]);
  }
  for (int k = 0; k < 2; ++k) a.drec[k] = tp<V4<T>>(F.drec[k]);
  // outgrown-list words by sub-step parity: this pass reads the word of its
  // positions and writes the word of the positions it produces
  if (pc.nbr && !rates_only) {
    pc.stale = c->S.stale + (c->substep & 1);
    a.stale_w = c->S.stale + ((c->substep + 1) & 1);
  } else {
    a.stale_w = nullptr;
    if (pc.nbr) pc.stale = c->S.stale + (c->substep & 1);
  }
  a.pid = F.pid.live();
  a.bufs = c->S.bufs;
  a.bidx = c->S.bidx;
  a.flags = c->S.flags;
  a.lrad = c->S.lrad;
  a.lskin = F.lskin;
  for (int k = 0; k < 3; ++k) a.cell_u[k] = tp<T>(F.cell_u[k]);
  a.t_el = (double)(c->substep + 1) * dt;
  a.dt = dt;
  a.step = c->step;
  a.t = c->t;
  a.rates_only = rates_only ? 1 : 0;
  a.o_ap = out ? out->ap : nullptr;
  if (rates_only) pc.pairs = nullptr;
  a.n_out = c->n_total;
  const int64_t n = c->n_total;
  const int L = team_lanes(c);
  switch (c->P.obc_mode) {
    case 1: SPHX_TEAM_SWITCH(L, launch_pass(c, &k_pressure<T, DIM, 1, TL>, nblk(n * TL), (int)n, pc, C, a)); break;
    case 2: SPHX_TEAM_SWITCH(L, launch_pass(c, &k_pressure<T, DIM, 2, TL>, nblk(n * TL), (int)n, pc, C, a)); break;
    case 3: SPHX_TEAM_SWITCH(L, launch_pass(c, &k_pressure<T, DIM, 3, TL>, nblk(n * TL), (int)n, pc, C, a)); break;
    default: SPHX_TEAM_SWITCH(L, launch_pass(c, &k_pressure<T, DIM, 4, TL>, nblk(n * TL), (int)n, pc, C, a)); break;
  }
  if (!rates_only)
    for (int k = 0; k < 3; ++k) {
      F.x[k].flip();
      F.xr[k].cur = F.x[k].cur;
    }
  return hipGetLastError();
}

template <typename T, int DIM>
hipError_t density_impl(sph_ctx* c, double dt, bool last, bool rates_only,
                        const sph_rates* out) {
  Consts<T> C = make_consts<T>(c);
  PairCtx<T> pc = make_pc<T>(c, c->F.xr, c->F.x[0].cur);
  if (pc.nbr) pc.stale = c->S.stale + (rates_only ? 0 : ((c->substep + 1) & 1));
  Fields& F = c->F;
  DensArgs<T> a;
  for (int k = 0; k < 3; ++k) a.v[k] = tp<T>(F.v[k].live());
  a.p = tp<T>(F.p.live());
  a.rho = F.rho.live();
  a.drho = tp<T>(F.drho.live());
  a.k = tp<T>(F.k.live());
  a.p_out = tp<T>(F.p.other());
  a.vol_out = tp<T>(F.vol.other());
  a.half_dt = 0.5 * dt;
  a.last = last ? 1 : 0;
  a.rates_only = rates_only ? 1 : 0;
  a.o_drho = out ? out->drho : nullptr;
  if (rates_only) pc.pairs = nullptr;
  for (int k = 0; k < 2; ++k) a.drec[k] = tp<V4<T>>(F.drec[k]);
  for (int k = 0; k < 3; ++k) a.prec[k] = tp<V4<T>>(F.prec[k]);
  for (int k = 0; k < 6; ++k) a.B[k] = tp<T>(F.B[k]);
  const int64_t n = c->n_total;
  const int L = team_lanes(c);
  if (c->P.turbulence) {
    SPHX_TEAM_SWITCH(L, launch_pass(c, &k_density<T, DIM, 1, TL>, nblk(n * TL), (int)n, pc, C, a));
  } else {
    SPHX_TEAM_SWITCH(L, launch_pass(c, &k_density<T, DIM, 0, TL>, nblk(n * TL), (int)n, pc, C, a));
  }
  if (!rates_only && !last) {
    F.p.flip();
    F.vol.flip();
  }
  return hipGetLastError();
}

template <typename T, int DIM>
hipError_t prepare_pv_impl(sph_ctx* c, const sph_rates* out) {
  Consts<T> C = make_consts<T>(c);
  Fields& F = c->F;
  F.p.cur = 0;
  F.vol.cur = 0;
  const int64_t n = c->n_total;
  PvArgs<T> a;
  a.rho = F.rho.live();
  a.k = tp<T>(F.k.live());
  a.tag = F.tag.live();
  a.p = tp<T>(F.p.live());
  a.vol = tp<T>(F.vol.live());
  a.o_p = out ? out->p : nullptr;
  for (int k = 0; k < 3; ++k) {
    a.xr[k] = tp<T>(F.xr[k].live());
    a.v[k] = tp<T>(F.v[k].live());
    a.prec[k] = tp<V4<T>>(F.prec[k]);
  }
  for (int k = 0; k < 6; ++k) a.B[k] = tp<T>(F.B[k]);
  for (int k = 0; k < 2; ++k) a.drec[k] = tp<V4<T>>(F.drec[k]);
  k_prepare_pv<T, DIM><<<nblk(n), 256, 0, c->stream>>>((int)n, C, a);
  return hipGetLastError();
}

template <typename T>
hipError_t reduce_impl(sph_ctx* c, double* host2, bool after_update, bool keys) {
  Fields& F = c->F;
  const int64_t n = c->n_total;
  const int64_t n_max = after_update ? std::min<int64_t>(c->cap, n + kMaxInject) : n;
  const int nb = nblk(n_max);
  if (after_update) {
    c->post_blocks = std::min(nb, kPostBlocks);
    KeyOut ko;
    for (int k = 0; k < 3; ++k) ko.x[k] = F.x[k].live();
    ko.g = c->grid;
    ko.key = keys ? c->S.key : nullptr;
    ko.slot = c->S.slot;
    ko.count = c->S.count;
    auto go = [&](auto dimtag) {
      constexpr int D = decltype(dimtag)::value;
      k_reduce_post<T, D><<<c->post_blocks, 256, 0, c->stream>>>(
          (int)n, (int)n_max, c->S.counters, tp<T>(F.v[0].live()), tp<T>(F.v[1].live()),
          tp<T>(F.v[2].live()), F.rho.live(), tp<T>(F.nut.live()), F.tag.live(),
          c->P.turbulence, c->S.flags, c->S.next_pid, (int)c->n_alive, c->S.nstate,
          c->pinned_dev, ko, c->S.stale);
    };
    if (c->P.dim == 2) go(std::integral_constant<int, 2>());
    else go(std::integral_constant<int, 3>());
    return hipGetLastError();
  }
  k_reduce_part<T><<<nb, 256, 0, c->stream>>>((int)n, after_update ? c->S.counters + 1024 : nullptr,
                                               (int)n_max, tp<T>(F.v[0].live()),
                                               tp<T>(F.v[1].live()), tp<T>(F.v[2].live()),
                                               F.rho.live(), tp<T>(F.nut.live()), F.tag.live(),
                                               c->P.turbulence, c->S.red + 4);
  k_reduce_final<<<1, 256, 0, c->stream>>>(nb, c->S.red + 4, c->S.red, c->S.flags);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !host2) return e;
  return hipMemcpyAsync(host2, c->S.red, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
}

template <typename T, int DIM>
hipError_t shift_apply_impl(sph_ctx* c) {
  Fields& F = c->F;
  const int64_t n = c->n_total;
  k_shift_apply<T, DIM><<<nblk(n), 256, 0, c->stream>>>(
      (int)n, F.tag.live(), tp<T>(F.shift[0]), tp<T>(F.shift[1]), tp<T>(F.shift[2]),
      F.x[0].live(), F.x[1].live(), F.x[2].live(), tp<T>(F.xr[0].live()),
      tp<T>(F.xr[1].live()), tp<T>(F.xr[2].live()));
  return hipGetLastError();
}

template <typename T, int DIM>
hipError_t walk_pairs_impl(sph_ctx* c, int32_t* row_ptr, int32_t* col, int64_t cap,
                           int64_t* n_pairs) {
  const int64_t n = c->n_total;
  PairCtx<T> pc = make_pc<T>(c, c->F.xr, c->F.x[0].cur);
  pc.pairs = nullptr;
  int32_t* counts = c->S.slot;   // scratch (rewritten by every cell build)
  k_walk_pairs<T, DIM, 0><<<nblk(n), 256, 0, c->stream>>>((int)n, pc, counts, col, cap);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_scan_excl(c, counts, (int)n, row_ptr);
  if (e != hipSuccess) return e;
  int32_t* total = reinterpret_cast<int32_t*>(c->pinned);
  e = hipMemcpyAsync(total, row_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return e;
  *n_pairs = *total;
  k_walk_pairs<T, DIM, 1><<<nblk(n), 256, 0, c->stream>>>((int)n, pc, row_ptr, col, cap);
  return hipGetLastError();
}

template <typename T, int DIM>
hipError_t export_B_impl(sph_ctx* c, double* B) {
  Fields& F = c->F;
  const int64_t n = c->n_total;
  k_export_B<T, DIM><<<nblk(n), 256, 0, c->stream>>>(
      (int)n, tp<T>(F.B[0]), tp<T>(F.B[1]), tp<T>(F.B[2]), tp<T>(F.B[3]), tp<T>(F.B[4]),
      tp<T>(F.B[5]), B);
  return hipGetLastError();
}

}  // namespace

#define SPHX_DISPATCH(fn, ...)                                                   \
  (c->P.precision == SPH_FP64                                                    \
       ? (c->P.dim == 2 ? fn<double, 2>(__VA_ARGS__) : fn<double, 3>(__VA_ARGS__)) \
       : (c->P.dim == 2 ? fn<float, 2>(__VA_ARGS__) : fn<float, 3>(__VA_ARGS__)))

hipError_t launch_correction(sph_ctx* c, const int32_t* ns, int64_t n_grid, bool tight,
                             bool moment) {
  c->B_pending = false;
  return SPHX_DISPATCH(correction_impl, c, ns, n_grid, tight, moment);
}

hipError_t launch_moment(sph_ctx* c) { return SPHX_DISPATCH(moment_impl, c, nullptr, c->n_total); }

hipError_t launch_advection(sph_ctx* c, double dt_adv, double dt_sub, bool rates_only,
                            const sph_rates* out) {
  return SPHX_DISPATCH(advection_impl, c, dt_adv, dt_sub, rates_only, out);
}

hipError_t launch_pressure(sph_ctx* c, double dt, bool rates_only, const sph_rates* out) {
  return SPHX_DISPATCH(pressure_impl, c, dt, rates_only, out);
}

hipError_t launch_density(sph_ctx* c, double dt, bool last, bool rates_only,
                          const sph_rates* out) {
  return SPHX_DISPATCH(density_impl, c, dt, last, rates_only, out);
}

hipError_t launch_prepare_pv(sph_ctx* c, const sph_rates* out) {
  return SPHX_DISPATCH(prepare_pv_impl, c, out);
}

hipError_t launch_reduce(sph_ctx* c, double* host2, bool after_update, bool keys) {
  return c->P.precision == SPH_FP64 ? reduce_impl<double>(c, host2, after_update, keys)
                                    : reduce_impl<float>(c, host2, after_update, keys);
}

hipError_t launch_export_B(sph_ctx* c, double* B) { return SPHX_DISPATCH(export_B_impl, c, B); }

hipError_t launch_list_dt(sph_ctx* c, bool fresh) {
  const sph_params& P = c->P;
  const double* part = reinterpret_cast<const double*>(c->pinned_dev + 1040);
  int nb = c->post_blocks;
  if (fresh) {   // the maxima of the current state (the same set of particles, exact maxima)
    hipError_t e = launch_reduce(c, nullptr, false, false);
    if (e != hipSuccess) return e;
    part = c->S.red + 4;
    nb = nblk(c->n_total);
  }
  k_list_dt<<<1, kListDtThreads, 0, c->stream>>>(nb, part, P.h, P.cfl_adv, P.u_ref, P.nu_l,
                                                 c->S.lrad);
  return hipGetLastError();
}

hipError_t launch_neighbors_noalloc(sph_ctx* c, int32_t* row_ptr, int32_t* col, int64_t cap,
                                    int64_t* n_pairs) {
  const int64_t n = c->n_total;
  int32_t* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (c->device >= 0 && c->device < kMaxDevices) base = g_scratch_dev[c->device];
  }
  if (!base || n > kNoAllocMaxN) return hipErrorInvalidValue;
  int32_t* counts = base;                  // [n]
  int32_t* part = base + kNoAllocMaxN;     // [kNoAllocParts]
  const double rc = 2.0 * c->P.h;
  const double rc2 = rc * rc;
  Fields& F = c->F;
  const int nb = nblk(n);
  auto go = [&](auto dimtag, auto filltag, int32_t* row) {
    constexpr int D = decltype(dimtag)::value;
    constexpr int FL = decltype(filltag)::value;
    k_neighbors<D, FL><<<nb, 256, 0, c->stream>>>(
        (int)n, F.x[0].live(), F.x[1].live(), F.x[2].live(), F.cell, c->S.cell_start,
        c->grid.n[0], c->grid.n[1], rc2, row, col, cap);
  };
  using D2 = std::integral_constant<int, 2>;
  using D3 = std::integral_constant<int, 3>;
  using F0 = std::integral_constant<int, 0>;
  using F1 = std::integral_constant<int, 1>;
  if (c->P.dim == 2) go(D2{}, F0{}, counts); else go(D3{}, F0{}, counts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_scan_excl_part(c, counts, (int)n, row_ptr, part);
  if (e != hipSuccess) return e;
  int32_t* total = reinterpret_cast<int32_t*>(c->pinned);   // the context's pinned buffer
  e = hipMemcpyAsync(total, row_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return e;
  *n_pairs = *total;
  if (c->P.dim == 2) go(D2{}, F1{}, row_ptr); else go(D3{}, F1{}, row_ptr);
  return hipGetLastError();
}

hipError_t launch_walk_pairs(sph_ctx* c, int32_t* row_ptr, int32_t* col, int64_t cap,
                             int64_t* n_pairs) {
  return SPHX_DISPATCH(walk_pairs_impl, c, row_ptr, col, cap, n_pairs);
}

hipError_t launch_shift_apply(sph_ctx* c) { return SPHX_DISPATCH(shift_apply_impl, c); }

hipError_t launch_neighbors(sph_ctx* c, int32_t* row_ptr, int32_t* col, int64_t cap,
                            int64_t* n_pairs) {
  const int64_t n = c->n_total;
  const double rc = 2.0 * c->P.h;
  const double rc2 = rc * rc;
  Fields& F = c->F;
  const int nb = nblk(n);
  auto go = [&](auto dimtag, auto filltag) {
    constexpr int D = decltype(dimtag)::value;
    constexpr int FL = decltype(filltag)::value;
    k_neighbors<D, FL><<<nb, 256, 0, c->stream>>>(
        (int)n, F.x[0].live(), F.x[1].live(), F.x[2].live(), F.cell, c->S.cell_start,
        c->grid.n[0], c->grid.n[1], rc2, row_ptr, col, cap);
  };
  using D2 = std::integral_constant<int, 2>;
  using D3 = std::integral_constant<int, 3>;
  using F1 = std::integral_constant<int, 1>;
  int32_t* counts = c->S.slot;   // scratch (rewritten by every cell build)
  auto go_count = [&](auto dimtag) {
    constexpr int D = decltype(dimtag)::value;
    k_neighbors<D, 0><<<nb, 256, 0, c->stream>>>(
        (int)n, F.x[0].live(), F.x[1].live(), F.x[2].live(), F.cell, c->S.cell_start,
        c->grid.n[0], c->grid.n[1], rc2, counts, col, cap);
  };
  if (c->P.dim == 2) go_count(D2{}); else go_count(D3{});
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_scan_excl(c, counts, (int)n, row_ptr);
  if (e != hipSuccess) return e;
  int32_t total = 0;
  e = hipMemcpyAsync(&total, row_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return e;
  *n_pairs = total;
  if (c->P.dim == 2) go(D2{}, F1{}); else go(D3{}, F1{});
  return hipGetLastError();
}

}  // namespace sphx
