// Inlet-profile sensitivity on gfx950: the objectives (slab mass flux, mean
// wall shear stress) and the discrete adjoint of one advection step of the
// laminar scheme with its buffer update, in FP64.
//
// The adjoint replays the step from its recorded start state with the
// recorded time step, buffer decisions and slab membership, keeping the
// sub-step states, then walks the step backwards:
//   buffer update (recycled parents and their copies, by particle id)
//   -> objective seeds -> for each acoustic sub-step in reverse:
//      continuity pass (Eqs. (discretize-continuity-equ-riemann),
//      (eq-intermediate-vel)) -> drift -> velocity boundary condition and
//      kick -> pressure pass (Eq. (eq-discretize-momentum-p-RKGC) with the
//      compensation of Eq. (eq-pressure-gradient-obc-B-final)) -> equation
//      of state -> viscous pass (Eq. (eq-discretize-momentum-ARD2), laminar)
//   -> correction matrix (Eq. (equ-B-matrix) with the mirror images of
//      Sec. 3.3, through the guarded inverse) -> volumes V = m / rho.
// Every pair pass is reversed in gather form: particle i collects the
// derivatives of its own sum and of its neighbours' sums with respect to its
// own variables, using the neighbours' cotangents computed beforehand, so
// there are no atomics and the result is deterministic.  The neighbour sets
// are those the forward pass evaluated (same positions, same predicate).
// The discrete events of the step (slab membership, mirror membership,
// decisions, the pair set at the cut-off) are held fixed: the kernel and its
// derivative vanish at the cut-off, so the pair set adds no terms.
#include <vector>

#include "sph_pairs.h"

namespace sphx {

hipError_t launch_buffer_forced(sph_ctx* c, const uint32_t* forced, uint32_t* log, int64_t pid_cap);

namespace {

inline int nblk_a(int64_t n) { return (int)((n + 255) / 256) + (n == 0); }

// f = W'(r) / r = kf (1 - q/2)^3 and its derivative f' = df/dr.
__device__ __forceinline__ void kernel_f(double r, double inv_h, double kf, double& f, double& fp) {
  const double t = 1.0 - 0.5 * r * inv_h;
  f = kf * t * t * t;
  fp = -1.5 * kf * inv_h * t * t;
}

// Reverse of a prescribed velocity v = u(y(x)) n_b (same factors as
// profile_speed): with c = n_b . lambda_v, adds c grad_x u to lx and, for the
// control buffer, c du/da_m to abar[m * stride] (the sine coefficients).
__device__ inline void bc_reverse(int dim, const BufDev& b, bool control, const double x[3],
                                  double c, uint64_t seed, uint32_t pid, int64_t step, double t,
                                  double lx[3], double* abar, int64_t stride) {
  double y[3];
  to_local(b, x[0], x[1], x[2], y);
  const double s = (y[1] + b.hw[0]) / (2.0 * b.hw[0]);
  double dFs = 0.0, dFt = 0.0;
  double fac = 1.0;
  if (b.noise_amp != 0.0) fac = 1.0 + b.noise_amp * counter_uniform(seed, pid, step, 0);
  fac *= buffer_ramp(b, t);
  if (b.profile == kProfParabolic) {
    double F = 4.0 * b.u0 * s * (1.0 - s);
    dFs = 4.0 * b.u0 * (1.0 - 2.0 * s);
    if (dim == 3) {
      const double tt = (y[2] + b.hw[1]) / (2.0 * b.hw[1]);
      const double G = 4.0 * tt * (1.0 - tt);
      dFt = F * 4.0 * (1.0 - 2.0 * tt);
      dFs *= G;
    }
  } else if (b.profile == kProfSine) {
    dFs = 4.0 * b.u0 * (1.0 - 2.0 * s);
    for (int m = 1; m <= b.n_coef; ++m) {
      const double a = (double)m * M_PI;
      double sn, cs;
      sincos(a * s, &sn, &cs);
      dFs += b.coef[m - 1] * a * cs;
      if (control) abar[(int64_t)(m - 1) * stride] += c * sn * fac;
    }
  }
  const double du1 = dFs * fac / (2.0 * b.hw[0]);
  const double du2 = dim == 3 ? dFt * fac / (2.0 * b.hw[1]) : 0.0;
  for (int k = 0; k < 3; ++k) lx[k] += c * (du1 * b.frame[3 + k] + du2 * b.frame[6 + k]);
}

// Frobenius product of two symmetric matrices in packed form.
template <int DIM>
__device__ __forceinline__ double sym_dot(const double a[6], const double b[6]) {
  double r = a[0] * b[0] + a[3] * b[3] + 2.0 * a[1] * b[1];
  if (DIM == 3) r += a[5] * b[5] + 2.0 * (a[2] * b[2] + a[4] * b[4]);
  return r;
}

// Packed symmetric product M = X S X (X, S symmetric).
template <int DIM>
__device__ __forceinline__ void sym_sandwich(const double X[6], const double S[6], double M[6]) {
  double Xf[3][3] = {{X[0], X[1], X[2]}, {X[1], X[3], X[4]}, {X[2], X[4], X[5]}};
  double Sf[3][3] = {{S[0], S[1], S[2]}, {S[1], S[3], S[4]}, {S[2], S[4], S[5]}};
  double T[3][3], R[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double s = 0.0;
      for (int k = 0; k < DIM; ++k) s += Xf[a][k] * Sf[k][b];
      T[a][b] = s;
    }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double s = 0.0;
      for (int k = 0; k < DIM; ++k) s += T[a][k] * Xf[k][b];
      R[a][b] = s;
    }
  M[0] = R[0][0]; M[1] = 0.5 * (R[0][1] + R[1][0]); M[3] = R[1][1];
  if (DIM == 3) {
    M[2] = 0.5 * (R[0][2] + R[2][0]); M[4] = 0.5 * (R[1][2] + R[2][1]); M[5] = R[2][2];
  } else {
    M[2] = M[4] = M[5] = 0.0;
  }
}

// Symmetric part of the outer product a b^T, packed, scaled by s, added to G.
template <int DIM>
__device__ __forceinline__ void add_sym_outer(double G[6], double s, const double a[3],
                                              const double b[3]) {
  G[0] += s * a[0] * b[0];
  G[1] += s * 0.5 * (a[0] * b[1] + a[1] * b[0]);
  G[3] += s * a[1] * b[1];
  if (DIM == 3) {
    G[2] += s * 0.5 * (a[0] * b[2] + a[2] * b[0]);
    G[4] += s * 0.5 * (a[1] * b[2] + a[2] * b[1]);
    G[5] += s * a[2] * b[2];
  }
}

template <int DIM>
__device__ __forceinline__ void symv_d(const double B[6], const double a[3], double o[3]) {
  if (DIM == 2) {
    o[0] = B[0] * a[0] + B[1] * a[1];
    o[1] = B[1] * a[0] + B[3] * a[1];
    o[2] = 0.0;
  } else {
    o[0] = B[0] * a[0] + B[1] * a[1] + B[2] * a[2];
    o[1] = B[1] * a[0] + B[3] * a[1] + B[4] * a[2];
    o[2] = B[2] * a[0] + B[4] * a[1] + B[5] * a[2];
  }
}

__device__ __forceinline__ double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// ---------------------------------------------------------------------------
// Device views of the adjoint workspace.
// ---------------------------------------------------------------------------
struct AdjDev {
  int n;                     // particle slots of the step
  int64_t cap;               // stride of the per-particle arrays
  int64_t pid_cap;
  const uint32_t* tag;       // tags during the step
  const uint32_t* pid;
  const int32_t* cell;
  const int32_t* cs;
  int nx, ny;
  double csz, rc2, inv_h, kf;
  const uint32_t* nbr;       // the step's neighbour list (NULL: scan the stencil)
  const int32_t* ncnt;       // entries per particle (kNbrNoList: overflowed, stencil)
  int nk;                    // entries the list holds per particle
  const uint32_t* stale;     // [2] outgrown-list words of the replayed step
  // snapshots
  double* X;                 // [(N+1)][3][cap]
  double* XR;                // [(N+1)][3][cap]
  double* V;                 // [(N+1)][3][cap]
  double* RH;                // [(N+1)][cap]
  double* P;                 // [N][cap]
  double* VOL;               // [N][cap]
  double* DD;                // [N][cap]
  double* rho0;              // [cap]
  double* vol0;              // [cap]
  const double* B[6];
  // cotangents
  double *lx[3], *lv[3], *lr, *lD, *lDpre, *lp, *lV, *lB[6], *la[3], *qb[3], *sb[3],
      *ab[3], *cb[6], *lV0;
  double* abar;              // [16][cap]
  int32_t* child;            // [cap] child slot -> particle id of the copy (-1: none)
  V4<double>* rec[5];        // [nmax][cap] packed records of the reverse pair passes
  uint32_t* flags;
};

__device__ __forceinline__ const double* snap3(const double* base, int64_t cap, int s, int k) {
  return base + ((int64_t)s * 3 + k) * cap;
}

template <int DIM>
__device__ __forceinline__ void stencil_of(const AdjDev& A, int i, int& cx, int& cy, int& cz) {
  const int c = A.cell[i];
  cx = c % A.nx;
  const int cyz = c / A.nx;
  cy = cyz % A.ny;
  cz = cyz / A.ny;
}

// Neighbours of i at the positions `xr` of a snapshot (the same pairs as the
// forward pass visited: the step's neighbour list while it covered every
// sub-step of the replay, else the cell stencil), team of L lanes.
template <int DIM, int L, typename Fn>
__device__ __forceinline__ void adj_neighbors(const AdjDev& A, const double* const xr[3], int i,
                                              int lane, Fn&& fn) {
  const double xi0 = xr[0][i], xi1 = xr[1][i], xi2 = DIM == 3 ? xr[2][i] : 0.0;
  const int cnt = (A.nbr && !(A.stale[0] | A.stale[1])) ? A.ncnt[i] : kNbrNoList;
  if (cnt <= A.nk) {   // an overflowed list: the stencil below
    constexpr int kG = kUnroll / list_vec<DIM, L, kUnroll>();   // groups per batch
    for (int g0 = 0; list_entry<DIM, L, kUnroll>(g0, lane, 0) < cnt; g0 += kG) {
      uint32_t e[kUnroll];
      list_batch<DIM, L, kUnroll>(A.nbr, A.cap, i, lane, g0, cnt, e);
      double q0[kUnroll], q1[kUnroll], q2[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int j = list_j<DIM, L>(e, u, list_entry<DIM, L, kUnroll>(g0, lane, u) < cnt);
        q0[u] = xr[0][j];
        q1[u] = xr[1][j];
        q2[u] = DIM == 3 ? xr[2][j] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        if (list_entry<DIM, L, kUnroll>(g0, lane, u) >= cnt) break;
        const int j = (int)(e[u] & kNbrIdxMask);
        double r[3];
        r[0] = (xi0 - q0[u]) + nbr_shift<double>(e[u], 0, A.csz);
        r[1] = (xi1 - q1[u]) + nbr_shift<double>(e[u], 1, A.csz);
        r[2] = DIM == 3 ? (xi2 - q2[u]) + nbr_shift<double>(e[u], 2, A.csz) : 0.0;
        const double r2 = DIM == 3 ? (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]
                                   : r[0] * r[0] + r[1] * r[1];
        if (r2 < A.rc2) fn(j, r, r2);
      }
    }
    return;
  }
  int cx, cy, cz;
  stencil_of<DIM>(A, i, cx, cy, cz);
  constexpr int zr = DIM == 3 ? 1 : 0;
  for (int dz = -zr; dz <= zr; ++dz)
    for (int dy = -1; dy <= 1; ++dy) {
      const int base = ((cz + dz) * A.ny + (cy + dy)) * A.nx + cx;
      const int j0 = A.cs[base - 1], j1 = A.cs[base], j2 = A.cs[base + 1], j3 = A.cs[base + 2];
      const double oy = -(double)dy * A.csz, oz = -(double)dz * A.csz;
      for (int j = j0 + lane; j < j3; j += L) {
        const double ox = j < j1 ? A.csz : (j < j2 ? 0.0 : -A.csz);
        double r[3];
        r[0] = (xi0 - xr[0][j]) + ox;
        r[1] = (xi1 - xr[1][j]) + oy;
        r[2] = DIM == 3 ? (xi2 - xr[2][j]) + oz : 0.0;
        const double r2 = DIM == 3 ? (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]
                                   : r[0] * r[0] + r[1] * r[1];
        if (r2 < A.rc2 && j != i) fn(j, r, r2);
      }
    }
}

// Packed j-side records of the reverse continuity and pressure passes
// (32-byte vectors of FP64), written per sub-step by the per-particle kernel
// that precedes each pass, so that a pass gathers NR vectors per candidate
// instead of a dozen scalars.  Flat value order (V negative for walls):
//   continuity: x[DIM], V, p, v[DIM], w = 2 rho lD
//   pressure:   x[DIM], V, p, B (2D: xx, xy, yy; 3D: xx, xy, xz, yy, yz, zz),
//               Q[DIM], s[DIM]
// The two sets are never live together and share storage.
template <int DIM>
struct AdjRec {
  static constexpr int iV = DIM, ip = DIM + 1;
  // continuity
  static constexpr int iv = DIM + 2, iw = 2 * DIM + 2, nd = (2 * DIM + 3 + 3) / 4;
  // pressure
  static constexpr int nB = DIM == 2 ? 3 : 6, iB = DIM + 2, iQ = iB + nB, is = iQ + DIM;
  static constexpr int np = (is + DIM + 3) / 4;
  static constexpr int nmax = np > nd ? np : nd;
};

template <int NR>
__device__ __forceinline__ void put_rec(V4<double>* const* rec, int i, const double (&v)[4 * NR]) {
#pragma unroll
  for (int w = 0; w < NR; ++w) rec[w][i] = V4<double>{v[4 * w], v[4 * w + 1], v[4 * w + 2], v[4 * w + 3]};
}

__device__ __forceinline__ double rv(const V4<double>* q, int k) {
  const V4<double>& v = q[k >> 2];
  switch (k & 3) {
    case 0: return v.a;
    case 1: return v.b;
    case 2: return v.c;
    default: return v.d;
  }
}

// The pairs of adj_neighbors over packed records (positions in the first
// DIM values): the NR vectors of every candidate of a batch are loaded
// before its tests; fn(j, r, r2, q) with q the records of j.
#ifndef SPHX_ADJ_UNROLL
#define SPHX_ADJ_UNROLL 2
#endif
template <int DIM, int L, int NR, typename Fn>
__device__ __forceinline__ void adj_neighbors_rec(const AdjDev& A, const V4<double>* const* rec,
                                                  int i, int lane, const double xi[3], Fn&& fn) {
  constexpr int U = SPHX_ADJ_UNROLL;
  const int cnt = (A.nbr && !(A.stale[0] | A.stale[1])) ? A.ncnt[i] : kNbrNoList;
  if (cnt <= A.nk) {   // an overflowed list: the stencil below
    constexpr int kG = U / list_vec<DIM, L, U>();   // groups per batch
    for (int g0 = 0; list_entry<DIM, L, U>(g0, lane, 0) < cnt; g0 += kG) {
      uint32_t e[U];
      list_batch<DIM, L, U>(A.nbr, A.cap, i, lane, g0, cnt, e);
      V4<double> q[U][NR];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = list_j<DIM, L>(e, u, list_entry<DIM, L, U>(g0, lane, u) < cnt);
#pragma unroll
        for (int w = 0; w < NR; ++w) q[u][w] = rec[w][j];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (list_entry<DIM, L, U>(g0, lane, u) >= cnt) break;
        const int j = (int)(e[u] & kNbrIdxMask);
        double r[3];
        r[0] = (xi[0] - q[u][0].a) + nbr_shift<double>(e[u], 0, A.csz);
        r[1] = (xi[1] - q[u][0].b) + nbr_shift<double>(e[u], 1, A.csz);
        r[2] = DIM == 3 ? (xi[2] - q[u][0].c) + nbr_shift<double>(e[u], 2, A.csz) : 0.0;
        const double r2 = DIM == 3 ? (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]
                                   : r[0] * r[0] + r[1] * r[1];
        if (r2 < A.rc2) fn(j, r, r2, q[u]);
      }
    }
    return;
  }
  int cx, cy, cz;
  stencil_of<DIM>(A, i, cx, cy, cz);
  constexpr int zr = DIM == 3 ? 1 : 0;
  for (int dz = -zr; dz <= zr; ++dz)
    for (int dy = -1; dy <= 1; ++dy) {
      const int base = ((cz + dz) * A.ny + (cy + dy)) * A.nx + cx;
      const int j0 = A.cs[base - 1], j1 = A.cs[base], j2 = A.cs[base + 1], j3 = A.cs[base + 2];
      const double oy = -(double)dy * A.csz, oz = -(double)dz * A.csz;
      for (int j = j0 + lane; j < j3; j += L) {
        V4<double> q[NR];
#pragma unroll
        for (int w = 0; w < NR; ++w) q[w] = rec[w][j];
        const double ox = j < j1 ? A.csz : (j < j2 ? 0.0 : -A.csz);
        double r[3];
        r[0] = (xi[0] - q[0].a) + ox;
        r[1] = (xi[1] - q[0].b) + oy;
        r[2] = DIM == 3 ? (xi[2] - q[0].c) + oz : 0.0;
        const double r2 = DIM == 3 ? (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]
                                   : r[0] * r[0] + r[1] * r[1];
        if (r2 < A.rc2 && j != i) fn(j, r, r2, q);
      }
    }
}

template <int L, int K>
__device__ __forceinline__ void team_sum_arr(double (&v)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = team_sum<L>(v[k]);
}

// ---------------------------------------------------------------------------
// Objectives (forward evaluation).
// ---------------------------------------------------------------------------
struct ObjArgs {
  double o[3], nrm[3], w, e[3], Lw;
  double m, mu, Vw;
  const double* x[3];
  const double* rho;
  const uint8_t* member_in;
  uint8_t* member_out;
  int64_t pid_cap;
  double* part;   // [2][nblocks]
};

__device__ __forceinline__ bool slab_member(const ObjArgs& a, double x0, double x1, double x2) {
  const double s = dadd(dadd(dmul(a.nrm[0], dsub(x0, a.o[0])), dmul(a.nrm[1], dsub(x1, a.o[1]))),
                        dmul(a.nrm[2], dsub(x2, a.o[2])));
  return s >= 0.0 && s < a.w;
}

template <typename T, int DIM>
__global__ __launch_bounds__(256) void k_objective(int n, PairCtx<T> pc, Consts<T> C,
                                                   const T* v0, const T* v1, const T* v2,
                                                   const uint32_t* pid, ObjArgs a) {
  __shared__ double sq[256], st[256];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double jq = 0.0, jt = 0.0;
  if (i < n && is_real(pc.tag[i])) {
    const uint32_t p = pid[i];
    const double vi[3] = {(double)v0[i], (double)v1[i], DIM == 3 ? (double)v2[i] : 0.0};
    bool in = a.member_in ? (p < a.pid_cap && a.member_in[p] != 0)
                          : slab_member(a, a.x[0][i], a.x[1][i], a.x[2][i]);
    if (a.member_out && p < a.pid_cap) a.member_out[p] = in ? 1 : 0;
    if (in) jq = a.m * dot3(a.nrm, vi) / a.w;
    const T xi[3] = {pc.xr[0][i], pc.xr[1][i], DIM == 3 ? pc.xr[2][i] : T(0)};
    double G = 0.0;
    for_neighbors<T, DIM, 1>(pc, i, 0, xi, [&](int j, const T r[3], T r2) {
      if (tag_kind(pc.tag[j]) == kWall) G += (double)dw_over_r<T>(sqrt(r2), C.inv_h_t, C.kf_t);
    });
    jt = -a.m * (2.0 / a.rho[i]) * a.mu * G * a.Vw * 2.0 * dot3(a.e, vi);
  }
  sq[threadIdx.x] = jq;
  st[threadIdx.x] = jt;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sq[threadIdx.x] += sq[threadIdx.x + o];
      st[threadIdx.x] += st[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.part[blockIdx.x] = sq[0];
    a.part[gridDim.x + blockIdx.x] = st[0];
  }
}

__global__ __launch_bounds__(256) void k_objective_final(int nb, const double* part, double Lw,
                                                         double* J) {
  __shared__ double sq[256], st[256];
  double q = 0.0, t = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) {
    q += part[b];
    t += part[nb + b];
  }
  sq[threadIdx.x] = q;
  st[threadIdx.x] = t;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sq[threadIdx.x] += sq[threadIdx.x + o];
      st[threadIdx.x] += st[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    J[0] += sq[0];
    J[1] += st[0] / Lw;
  }
}

__global__ void k_fill_u8(int64_t n, uint8_t* p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// ---------------------------------------------------------------------------
// Snapshots: up to 8 FP64 arrays copied in one launch.
// ---------------------------------------------------------------------------
// Snapshot copies into FP64; a source in the pair precision of an
// FP32-mixed forward (f32 set) is widened on the way.
struct CopyList {
  const void* src[10];
  double* dst[10];
  int f32[10];
  int k;
};

__global__ __launch_bounds__(256) void k_copy(int n, CopyList c) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int q = 0; q < c.k; ++q)
    c.dst[q][i] = c.f32[q] ? (double)static_cast<const float*>(c.src[q])[i]
                           : static_cast<const double*>(c.src[q])[i];
}

__global__ void k_copy_u32(int n, const uint32_t* s, uint32_t* d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = s[i];
}

// ---------------------------------------------------------------------------
// Reverse of the buffer update: the cotangent of the state before the update
// from the one after it (by particle id).  Deleted particles get zero; a
// recycled parent gets the reverse of the shift (identity) and of its
// boundary values, plus the cotangent of its copy.
// ---------------------------------------------------------------------------
struct PostArgs {
  const double* lam;        // [8][pid_cap]
  const uint32_t* dec;      // decisions by slot
  const BufDev* bufs;
  const int32_t* bidx;
  int control_q;
  int dim;
  uint64_t seed;
  int64_t step_post;
  double t_post;
};

__global__ __launch_bounds__(256) void k_adj_post(AdjDev A, PostArgs a, int N) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  const int64_t cap = A.cap;
  double l[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const uint32_t ti = A.tag[i];
  const uint32_t d = a.dec[i];
  const uint32_t act = d & 0xFFu;
  if (is_real(ti) && act != kDecDelete) {
    const uint32_t p = A.pid[i];
    if (p >= A.pid_cap) {
      atomicOr(A.flags, kFlagCapacity);
      return;
    }
    for (int k = 0; k < 8; ++k) l[k] = a.lam[(int64_t)k * A.pid_cap + p];
    if (act == kDecInject) {
      const int q = a.bidx[(d >> 8) & 0xFFu];
      const BufDev& b = a.bufs[q];
      if (b.vel_mode == kVelPrescribed) {
        double xn[3];
        for (int k = 0; k < 3; ++k)
          xn[k] = __dsub_rn(snap3(A.X, cap, N, k)[i], __dmul_rn(b.length, b.frame[k]));
        const double c = b.frame[0] * l[3] + b.frame[1] * l[4] + b.frame[2] * l[5];
        bc_reverse(a.dim, b, q == a.control_q, xn, c, a.seed, p, a.step_post, a.t_post, l,
                   A.abar + i, cap);
        l[3] = l[4] = l[5] = 0.0;
      }
      if (b.p_mode == kPPrescribed) l[6] = 0.0;
      const int cp = A.child[i];
      if (cp < 0 || cp >= A.pid_cap) {
        atomicOr(A.flags, kFlagCapacity);
      } else {
        for (int k = 0; k < 8; ++k) l[k] += a.lam[(int64_t)k * A.pid_cap + cp];
      }
    }
  }
  for (int k = 0; k < 3; ++k) {
    A.lx[k][i] = l[k];
    A.lv[k][i] = l[3 + k];
  }
  A.lr[i] = l[6];
  A.lD[i] = l[7];
}

__global__ __launch_bounds__(256) void k_adj_children(AdjDev A, const int32_t* inj,
                                                      uint64_t base_pid) {
  // inj[0]: injections of the update, inj[1 + r]: parent slot of child r
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int m = inj[0];
  const int32_t* inj_idx = inj + 1;
  if (r >= m || r >= kMaxInject) return;
  const int i = inj_idx[r];
  if (i >= 0 && i < A.n) A.child[i] = (int32_t)(base_pid + (uint64_t)r);
}

__global__ void k_fill_child(int n, int32_t* child) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) child[i] = -1;
}

// ---------------------------------------------------------------------------
// Objective seeds at the state after the step (i-local; walls are fixed).
// ---------------------------------------------------------------------------
struct SeedArgs {
  const uint8_t* member;
  double wq, wt;
  double nrm[3], w, e[3], Lw, m, mu, Vw;
};

template <int DIM, int L>
__global__ __launch_bounds__(256) void k_adj_seed(AdjDev A, SeedArgs s, int N) {
  const int g = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int i = g / L, lane = g % L;
  if (i >= A.n) return;
  if (!is_real(A.tag[i])) return;
  const int64_t cap = A.cap;
  const double* xr[3] = {snap3(A.XR, cap, N, 0), snap3(A.XR, cap, N, 1), snap3(A.XR, cap, N, 2)};
  double acc[4] = {0, 0, 0, 0};   // sum f, sum f' r_hat
  if (s.wt != 0.0) {
    adj_neighbors<DIM, L>(A, xr, i, lane, [&](int j, const double r[3], double r2) {
      if (tag_kind(A.tag[j]) != kWall) return;
      const double rr = sqrt(r2);
      double f, fp;
      kernel_f(rr, A.inv_h, A.kf, f, fp);
      acc[0] += f;
      for (int k = 0; k < 3; ++k) acc[1 + k] += fp * r[k] / rr;
    });
    team_sum_arr<L>(acc);
  }
  if (lane != 0) return;
  const double vi[3] = {snap3(A.V, cap, N, 0)[i], snap3(A.V, cap, N, 1)[i],
                        DIM == 3 ? snap3(A.V, cap, N, 2)[i] : 0.0};
  const uint32_t p = A.pid[i];
  if (s.member && p < A.pid_cap && s.member[p])
    for (int k = 0; k < DIM; ++k) A.lv[k][i] += s.wq * s.m * s.nrm[k] / s.w;
  if (s.wt != 0.0) {
    const double rho = A.RH[(int64_t)N * cap + i];
    const double c = s.m * 2.0 * s.mu * s.Vw * 2.0 / s.Lw;
    const double ve = dot3(s.e, vi);
    for (int k = 0; k < DIM; ++k) {
      A.lv[k][i] += s.wt * (-c * acc[0] / rho) * s.e[k];
      A.lx[k][i] += s.wt * (-c * ve / rho) * acc[1 + k];
    }
    A.lr[i] += s.wt * c * ve * acc[0] / (rho * rho);
  }
}

// ---------------------------------------------------------------------------
// Continuity pass of sub-step s (positions x_{s+1}, velocities v_{s+1},
// p_s, V_s, rho_h,s):  D_i = 2 rho_i sum_j V_j f (v_ij . r / 2 + kappa p_ij |r|)
// with walls v_j = 0, p_j = p_i; kappa = 1 / (2 rho0 c0).
// ---------------------------------------------------------------------------
// Continuity record of particle i for the reverse pass of sub-step s
// (positions and velocities after the sub-step, p and V at it).
template <int DIM>
__device__ __forceinline__ void put_drec(const AdjDev& A, int i, int s, double lD) {
  using R = AdjRec<DIM>;
  const int64_t cap = A.cap;
  double v[4 * R::nd];
#pragma unroll
  for (int k = 0; k < 4 * R::nd; ++k) v[k] = 0.0;
  const uint32_t t = A.tag[i];
  const double vol = A.VOL[(int64_t)s * cap + i];
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    v[k] = snap3(A.XR, cap, s + 1, k)[i];
    v[R::iv + k] = snap3(A.V, cap, s + 1, k)[i];
  }
  v[R::iV] = tag_kind(t) == kWall ? -vol : vol;
  v[R::ip] = A.P[(int64_t)s * cap + i];
  v[R::iw] = is_real(t) ? 2.0 * A.RH[(int64_t)s * cap + i] * lD : 0.0;
  put_rec<R::nd>(A.rec, i, v);
}

// Pressure record of particle i for the reverse pass of sub-step s, with
// the cotangents Q and s of the kick.
template <int DIM>
__device__ __forceinline__ void put_prec_adj(const AdjDev& A, int i, int s, const double Q[3],
                                             const double sv[3]) {
  using R = AdjRec<DIM>;
  const int64_t cap = A.cap;
  double v[4 * R::np];
#pragma unroll
  for (int k = 0; k < 4 * R::np; ++k) v[k] = 0.0;
  const double vol = A.VOL[(int64_t)s * cap + i];
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    v[k] = snap3(A.XR, cap, s, k)[i];
    v[R::iQ + k] = Q[k];
    v[R::is + k] = sv[k];
  }
  v[R::iV] = tag_kind(A.tag[i]) == kWall ? -vol : vol;
  v[R::ip] = A.P[(int64_t)s * cap + i];
  if (DIM == 2) {
    v[R::iB] = A.B[0][i];
    v[R::iB + 1] = A.B[1][i];
    v[R::iB + 2] = A.B[3][i];
  } else {
#pragma unroll
    for (int k = 0; k < 6; ++k) v[R::iB + k] = A.B[k][i];
  }
  put_rec<R::np>(A.rec, i, v);
}

template <int DIM>
__global__ __launch_bounds__(256) void k_adj_dprep(AdjDev A, int last, double half, int s) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  double lD = 0.0;
  if (is_real(A.tag[i])) {
    // last sub-step: D_{N-1} is the carried rate, rho_end = rho_h + dt/2 D;
    // earlier: rho_h,s+1 = rho_h,s + dt D_s
    lD = last ? A.lD[i] + half * A.lr[i] : 2.0 * half * A.lr[i];
  }
  A.lD[i] = lD;
  put_drec<DIM>(A, i, s, lD);
}

template <int DIM, int L>
__global__ __launch_bounds__(256) void k_adj_density(AdjDev A, int s, double kappa) {
  const int g = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int i = g / L, lane = g % L;
  if (i >= A.n) return;
  if (!is_real(A.tag[i])) return;
  const int64_t cap = A.cap;
  using R = AdjRec<DIM>;
  const double xi[3] = {snap3(A.XR, cap, s + 1, 0)[i], snap3(A.XR, cap, s + 1, 1)[i],
                        DIM == 3 ? snap3(A.XR, cap, s + 1, 2)[i] : 0.0};
  const double vi[3] = {snap3(A.V, cap, s + 1, 0)[i], snap3(A.V, cap, s + 1, 1)[i],
                        DIM == 3 ? snap3(A.V, cap, s + 1, 2)[i] : 0.0};
  const double* rh = A.RH + (int64_t)s * cap;
  const double pi = A.P[(int64_t)s * cap + i], Vi = A.VOL[(int64_t)s * cap + i];
  const double wi = 2.0 * rh[i] * A.lD[i];
  // lv[3], lx[3], lp, lV
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  adj_neighbors_rec<DIM, L, R::nd>(A, A.rec, i, lane, xi,
                                   [&](int j, const double r[3], double r2, const V4<double>* q) {
    const double rr = sqrt(r2);
    double f, fp;
    kernel_f(rr, A.inv_h, A.kf, f, fp);
    const double rh_[3] = {r[0] / rr, r[1] / rr, r[2] / rr};
    const double Vs = rv(q, R::iV);
    const double Vj = Vs < 0.0 ? -Vs : Vs;
    if (Vs < 0.0) {   // wall
      const double Sij = 0.5 * dot3(vi, r);
      for (int k = 0; k < DIM; ++k) {
        acc[k] += 0.5 * f * r[k] * wi * Vj;
        acc[3 + k] += wi * Vj * (fp * rh_[k] * Sij + f * 0.5 * vi[k]);
      }
      return;
    }
    const double wj = rv(q, R::iw);
    const double vij[3] = {vi[0] - rv(q, R::iv), vi[1] - rv(q, R::iv + 1),
                           DIM == 3 ? vi[2] - rv(q, R::iv + 2) : 0.0};
    const double pij = pi - rv(q, R::ip);
    const double Sij = 0.5 * dot3(vij, r) + kappa * pij * rr;
    const double Sji = 0.5 * dot3(vij, r) - kappa * pij * rr;
    for (int k = 0; k < DIM; ++k) {
      acc[k] += 0.5 * f * r[k] * (wi * Vj + wj * Vi);
      acc[3 + k] += wi * Vj * (fp * rh_[k] * Sij + f * (0.5 * vij[k] + kappa * pij * rh_[k])) +
                    wj * Vi * (fp * rh_[k] * Sji + f * (0.5 * vij[k] - kappa * pij * rh_[k]));
    }
    acc[6] += kappa * f * rr * (wi * Vj - wj * Vi);
    acc[7] += wj * f * Sji;
  });
  team_sum_arr<L>(acc);
  if (lane != 0) return;
  for (int k = 0; k < DIM; ++k) {
    A.lv[k][i] += acc[k];
    A.lx[k][i] += acc[3 + k];
  }
  A.lp[i] += acc[6];
  A.lV[i] += acc[7];
  A.lr[i] += A.lD[i] * A.DD[(int64_t)s * cap + i] / rh[i];
}

// ---------------------------------------------------------------------------
// Drift, velocity boundary condition and kick of sub-step s (i-local):
// x_{s+1} = x_s + dt v_{s+1};  v_{s+1} = u(y(x_s)) n_b (prescribed buffer
// particles) or v_s + dt (a_p + a_nu + g).  Also the cotangents that the
// pressure pass needs from every particle: Qbar = -dt lv / rho and the
// compensation's sbar = -2 p_ob (B Qbar | Qbar).
// ---------------------------------------------------------------------------
struct KickArgs {
  const BufDev* bufs;
  const int32_t* bidx;
  int control_q, dim, mode;
  uint64_t seed;
  int64_t step;
  double t, dt;
};

template <int DIM>
__global__ __launch_bounds__(256) void k_adj_kick(AdjDev A, KickArgs a, int s) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  const double zero[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < 3; ++k) {
    A.qb[k][i] = 0.0;
    A.sb[k][i] = 0.0;
  }
  const uint32_t ti = A.tag[i];
  if (!is_real(ti)) {
    put_prec_adj<DIM>(A, i, s, zero, zero);
    return;
  }
  const int64_t cap = A.cap;
  double lv[3], lx[3];
  for (int k = 0; k < 3; ++k) {
    lx[k] = A.lx[k][i];
    lv[k] = A.lv[k][i] + (k < DIM ? a.dt * lx[k] : 0.0);   // drift
  }
  int q = -1;
  if (tag_kind(ti) == kBuffer) q = a.bidx[tag_bid(ti)];
  if (q >= 0 && a.bufs[q].vel_mode == kVelPrescribed) {
    const BufDev& b = a.bufs[q];
    const double xs[3] = {snap3(A.X, cap, s, 0)[i], snap3(A.X, cap, s, 1)[i],
                          snap3(A.X, cap, s, 2)[i]};
    const double c = b.frame[0] * lv[0] + b.frame[1] * lv[1] + b.frame[2] * lv[2];
    bc_reverse(a.dim, b, q == a.control_q, xs, c, a.seed, A.pid[i], a.step, a.t, lx, A.abar + i,
               cap);
    for (int k = 0; k < 3; ++k) {
      A.lx[k][i] = lx[k];
      A.lv[k][i] = 0.0;
    }
    put_prec_adj<DIM>(A, i, s, zero, zero);
    return;
  }
  const double rho = A.RH[(int64_t)s * cap + i];
  double Qb[3];
  for (int k = 0; k < 3; ++k) {
    const double la = k < DIM ? a.dt * lv[k] : 0.0;
    A.la[k][i] += la;
    Qb[k] = -la / rho;
    A.qb[k][i] = Qb[k];
    A.lv[k][i] = lv[k];
  }
  double sv[3] = {0.0, 0.0, 0.0};
  if (q >= 0 && a.bufs[q].p_mode != kPNone) {
    const BufDev& b = a.bufs[q];
    const double pob = b.p_mode == kPPrescribed ? b.p_ob * buffer_ramp(b, a.t)
                                                : A.P[(int64_t)s * cap + i];
    double c[3];
    if (a.mode == 4) {
      double Bi[6];
      for (int k = 0; k < 6; ++k) Bi[k] = A.B[k][i];
      if (DIM == 2) Bi[2] = Bi[4] = Bi[5] = 0.0;
      symv_d<DIM>(Bi, Qb, c);
    } else {
      c[0] = Qb[0]; c[1] = Qb[1]; c[2] = Qb[2];
    }
    for (int k = 0; k < 3; ++k) {
      sv[k] = -2.0 * pob * c[k];
      A.sb[k][i] = sv[k];
    }
  }
  put_prec_adj<DIM>(A, i, s, Qb, sv);
}

// ---------------------------------------------------------------------------
// Pressure pass of sub-step s (positions x_s, p_s, V_s, rho_h,s, B):
// Q_i = sum_j V_j f M_ij r - 2 p_ob c_i,  M_ij = p_i B_j + p_j B_i (MODE >= 2)
// or (p_i + p_j) I (MODE 1); walls p_j = p_i, B_j = B_i; a_p = -Q / rho.
// ---------------------------------------------------------------------------
template <int DIM, int MODE, int L>
__global__ __launch_bounds__(256) void k_adj_pressure(AdjDev A, KickArgs a, int s) {
  const int g = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int i = g / L, lane = g % L;
  if (i >= A.n) return;
  const uint32_t ti = A.tag[i];
  if (!is_real(ti)) return;
  const int64_t cap = A.cap;
  using R = AdjRec<DIM>;
  const double xi[3] = {snap3(A.XR, cap, s, 0)[i], snap3(A.XR, cap, s, 1)[i],
                        DIM == 3 ? snap3(A.XR, cap, s, 2)[i] : 0.0};
  const double pi = A.P[(int64_t)s * cap + i], Vi = A.VOL[(int64_t)s * cap + i];
  double Bi[6] = {1, 0, 0, 1, 0, DIM == 3 ? 1.0 : 0.0};
  if (MODE >= 2)
    for (int k = 0; k < 6; ++k) Bi[k] = DIM == 2 && (k == 2 || k == 4 || k == 5) ? 0.0 : A.B[k][i];
  const double Qi[3] = {A.qb[0][i], A.qb[1][i], A.qb[2][i]};
  const double si_[3] = {A.sb[0][i], A.sb[1][i], A.sb[2][i]};
  // 0-2 lx, 3 lp, 4 lV, 5-10 lB, 11-13 Q (forward sum), 14-16 s (forward sum)
  double acc[17] = {0};
  adj_neighbors_rec<DIM, L, R::np>(A, A.rec, i, lane, xi,
                                   [&](int j, const double r[3], double r2, const V4<double>* q) {
    const double rr = sqrt(r2);
    double f, fp;
    kernel_f(rr, A.inv_h, A.kf, f, fp);
    const double rh_[3] = {r[0] / rr, r[1] / rr, r[2] / rr};
    const double Vs = rv(q, R::iV);
    const double Vj = Vs < 0.0 ? -Vs : Vs;
    const bool wall = Vs < 0.0;
    // s_i = sum_j V_j f r and the i- and j-side terms of sbar
    const double sj_[3] = {wall ? 0.0 : rv(q, R::is), wall ? 0.0 : rv(q, R::is + 1),
                           (wall || DIM == 2) ? 0.0 : rv(q, R::is + 2)};
    for (int k = 0; k < 3; ++k) acc[14 + k] += Vj * f * r[k];
    {
      const double di = dot3(si_, r), dj = dot3(sj_, r);
      for (int k = 0; k < DIM; ++k)
        acc[k] += Vj * (fp * rh_[k] * di + f * si_[k]) - Vi * (fp * rh_[k] * dj + f * sj_[k]);
      if (!wall) acc[4] += -f * dj;
    }
    if (wall) {
      double Mr[3], MQ[3];
      if (MODE >= 2) {
        double Bir[3];
        symv_d<DIM>(Bi, r, Bir);
        for (int k = 0; k < 3; ++k) Mr[k] = 2.0 * pi * Bir[k];
        symv_d<DIM>(Bi, Qi, MQ);
        for (int k = 0; k < 3; ++k) MQ[k] *= 2.0 * pi;
        acc[3] += 2.0 * Vj * f * dot3(Bir, Qi);
        add_sym_outer<DIM>(acc + 5, 2.0 * Vj * f * pi, Qi, r);
      } else {
        for (int k = 0; k < 3; ++k) {
          Mr[k] = 2.0 * pi * r[k];
          MQ[k] = 2.0 * pi * Qi[k];
        }
        acc[3] += 2.0 * Vj * f * dot3(r, Qi);
      }
      const double qm = dot3(Qi, Mr);
      for (int k = 0; k < DIM; ++k) acc[k] += Vj * (fp * rh_[k] * qm + f * MQ[k]);
      for (int k = 0; k < 3; ++k) acc[11 + k] += Vj * f * Mr[k];
      return;
    }
    const double pj = rv(q, R::ip);
    const double Qj[3] = {rv(q, R::iQ), rv(q, R::iQ + 1), DIM == 3 ? rv(q, R::iQ + 2) : 0.0};
    double Mr[3], MQi[3], MQj[3];
    if (MODE >= 2) {
      double Bj[6];
      if (DIM == 2) {
        Bj[0] = rv(q, R::iB);
        Bj[1] = rv(q, R::iB + 1);
        Bj[3] = rv(q, R::iB + 2);
        Bj[2] = Bj[4] = Bj[5] = 0.0;
      } else {
        for (int k = 0; k < 6; ++k) Bj[k] = rv(q, R::iB + k);
      }
      double Bjr[3], Bir[3], BjQi[3], BiQi[3], BjQj[3], BiQj[3];
      symv_d<DIM>(Bj, r, Bjr);
      symv_d<DIM>(Bi, r, Bir);
      symv_d<DIM>(Bj, Qi, BjQi);
      symv_d<DIM>(Bi, Qi, BiQi);
      symv_d<DIM>(Bj, Qj, BjQj);
      symv_d<DIM>(Bi, Qj, BiQj);
      for (int k = 0; k < 3; ++k) {
        Mr[k] = pi * Bjr[k] + pj * Bir[k];
        MQi[k] = pi * BjQi[k] + pj * BiQi[k];
        MQj[k] = pi * BjQj[k] + pj * BiQj[k];
      }
      acc[3] += f * (Vj * dot3(Bjr, Qi) - Vi * dot3(Bjr, Qj));
      double dq[3];
      for (int k = 0; k < 3; ++k) dq[k] = Vj * Qi[k] - Vi * Qj[k];
      add_sym_outer<DIM>(acc + 5, f * pj, dq, r);
    } else {
      for (int k = 0; k < 3; ++k) {
        Mr[k] = (pi + pj) * r[k];
        MQi[k] = (pi + pj) * Qi[k];
        MQj[k] = (pi + pj) * Qj[k];
      }
      acc[3] += f * (Vj * dot3(r, Qi) - Vi * dot3(r, Qj));
    }
    const double qi = dot3(Qi, Mr), qj = dot3(Qj, Mr);
    for (int k = 0; k < DIM; ++k)
      acc[k] += Vj * (fp * rh_[k] * qi + f * MQi[k]) - Vi * (fp * rh_[k] * qj + f * MQj[k]);
    acc[4] += -f * qj;
    for (int k = 0; k < 3; ++k) acc[11 + k] += Vj * f * Mr[k];
  });
  team_sum_arr<L>(acc);
  if (lane != 0) return;
  // compensation: Q_i -= 2 p_ob c_i, c_i = B_i s_i (MODE 4) or s_i
  const double rho = A.RH[(int64_t)s * cap + i];
  double Q[3] = {acc[11], acc[12], acc[13]};
  int q = -1;
  if (tag_kind(ti) == kBuffer) q = a.bidx[tag_bid(ti)];
  double lp = acc[3];
  double lB[6] = {acc[5], acc[6], acc[7], acc[8], acc[9], acc[10]};
  if (q >= 0 && a.bufs[q].p_mode != kPNone) {
    const BufDev& b = a.bufs[q];
    const double pob = b.p_mode == kPPrescribed ? b.p_ob * buffer_ramp(b, a.t) : pi;
    const double sv[3] = {acc[14], acc[15], acc[16]};
    double c[3];
    if (MODE == 4) symv_d<DIM>(Bi, sv, c);
    else { c[0] = sv[0]; c[1] = sv[1]; c[2] = sv[2]; }
    for (int k = 0; k < 3; ++k) Q[k] -= 2.0 * pob * c[k];
    if (b.p_mode == kPExtrapolate) lp += -2.0 * dot3(c, Qi);
    if (MODE == 4) add_sym_outer<DIM>(lB, -2.0 * pob, Qi, sv);
  }
  for (int k = 0; k < DIM; ++k) A.lx[k][i] += acc[k];
  A.lp[i] += lp;
  A.lV[i] += acc[4];
  if (MODE >= 2)
    for (int k = 0; k < 6; ++k) A.lB[k][i] += lB[k];
  A.lr[i] += -dot3(Qi, Q) / rho;
}

// Equation of state and volume of sub-step s: p = c0^2 (rho - rho0),
// V = m / rho (real particles), then the two-half-step density update back
// to the previous sub-step (identity in rho; the rate part is taken by
// k_adj_dprep of the previous sub-step).
__global__ __launch_bounds__(256) void k_adj_eos(AdjDev A, int s, double c02, double mass) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  if (is_real(A.tag[i])) {
    const double r = A.RH[(int64_t)s * A.cap + i];
    A.lr[i] += c02 * A.lp[i] - mass / (r * r) * A.lV[i];
  }
  A.lp[i] = 0.0;
  A.lV[i] = 0.0;
}

// k_adj_eos of sub-step s + 1 followed by k_adj_dprep of sub-step s (both
// per particle, one launch).
template <int DIM>
__global__ __launch_bounds__(256) void k_adj_eos_dprep(AdjDev A, int s1, double c02, double mass,
                                                       double half) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  double lD = 0.0;
  if (is_real(A.tag[i])) {
    const double r = A.RH[(int64_t)s1 * A.cap + i];
    const double lr = A.lr[i] + c02 * A.lp[i] - mass / (r * r) * A.lV[i];
    A.lr[i] = lr;
    lD = 2.0 * half * lr;
  }
  A.lp[i] = 0.0;
  A.lV[i] = 0.0;
  A.lD[i] = lD;
  put_drec<DIM>(A, i, s1 - 1, lD);
}

// ---------------------------------------------------------------------------
// Viscous pass (laminar; positions x_0, v_0, V^0, rho_0):
// a_nu,i = (2 mu / rho_i) sum_j f V_j v_ij, walls v_ij = 2 v_i.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_adj_vprep(AdjDev A, double two_mu, double half) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  // rho_h,0 = rho_0 + dt/2 D_pre
  A.lDpre[i] = is_real(A.tag[i]) ? half * A.lr[i] : 0.0;
  for (int k = 0; k < 3; ++k) A.ab[k][i] = is_real(A.tag[i]) ? two_mu / A.rho0[i] * A.la[k][i] : 0.0;
}

template <int DIM, int L>
__global__ __launch_bounds__(256) void k_adj_viscous(AdjDev A) {
  const int g = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int i = g / L, lane = g % L;
  if (i >= A.n) return;
  if (!is_real(A.tag[i])) return;
  const int64_t cap = A.cap;
  const double* xr[3] = {snap3(A.XR, cap, 0, 0), snap3(A.XR, cap, 0, 1), snap3(A.XR, cap, 0, 2)};
  const double* v[3] = {snap3(A.V, cap, 0, 0), snap3(A.V, cap, 0, 1), snap3(A.V, cap, 0, 2)};
  const double vi[3] = {v[0][i], v[1][i], DIM == 3 ? v[2][i] : 0.0};
  const double Vi = A.vol0[i];
  const double Ai[3] = {A.ab[0][i], A.ab[1][i], A.ab[2][i]};
  // 0-2 lv, 3-5 lx, 6 lV0, 7-9 U (forward sum)
  double acc[10] = {0};
  adj_neighbors<DIM, L>(A, xr, i, lane, [&](int j, const double r[3], double r2) {
    const double rr = sqrt(r2);
    double f, fp;
    kernel_f(rr, A.inv_h, A.kf, f, fp);
    const double Vj = A.vol0[j];
    if (tag_kind(A.tag[j]) == kWall) {
      const double q = 2.0 * dot3(Ai, vi);
      for (int k = 0; k < DIM; ++k) {
        acc[k] += 2.0 * f * Vj * Ai[k];
        acc[3 + k] += fp * r[k] / rr * Vj * q;
        acc[7 + k] += f * Vj * 2.0 * vi[k];
      }
      return;
    }
    const double Aj[3] = {A.ab[0][j], A.ab[1][j], A.ab[2][j]};
    const double vij[3] = {vi[0] - v[0][j], vi[1] - v[1][j], DIM == 3 ? vi[2] - v[2][j] : 0.0};
    const double qi = dot3(Ai, vij), qj = dot3(Aj, vij);
    for (int k = 0; k < DIM; ++k) {
      acc[k] += f * (Vj * Ai[k] - Vi * Aj[k]);
      acc[3 + k] += fp * r[k] / rr * (Vj * qi - Vi * qj);
      acc[7 + k] += f * Vj * vij[k];
    }
    acc[6] += -f * qj;
  });
  team_sum_arr<L>(acc);
  if (lane != 0) return;
  for (int k = 0; k < DIM; ++k) {
    A.lv[k][i] += acc[k];
    A.lx[k][i] += acc[3 + k];
  }
  A.lV0[i] += acc[6];
  const double U[3] = {acc[7], acc[8], acc[9]};
  A.lr[i] += -dot3(Ai, U) / A.rho0[i];
}

// ---------------------------------------------------------------------------
// Correction matrix: A_i = -sum_j V_j f r r^T (+ mirror images of real j for
// i within 2h of an open face), B_i = guarded inverse of A_i.
// ---------------------------------------------------------------------------
struct CorrAdjArgs {
  const double* x[3];   // FP64 positions x_0
  const BufDev* bufs;
  int nbuf, mirror;
  double twoh;
  GridDev grid;
};

// Mirror images of real j across buffer b's open face within the cut-off of
// the point (xi), i in [0, 2h) of the face: calls fn(j, r') with
// r' = x_i - (x_j - 2 y_j0 n_b), as the forward correction pass forms it.
template <int DIM, int L, typename Fn>
__device__ __forceinline__ bool mirror_partners(const AdjDev& A, const CorrAdjArgs& c,
                                                const BufDev& b, const double xi[3], int lane,
                                                bool want_i_side, Fn&& fn) {
  // the search centre: the image of i (i-side) is where its partners' images sit
  double yi[3];
  to_local(b, xi[0], xi[1], xi[2], yi);
  const double tt = 2.0 * yi[0];
  const double m[3] = {xi[0] - tt * b.frame[0], xi[1] - tt * b.frame[1], xi[2] - tt * b.frame[2]};
  int cm[3] = {0, 0, 0};
  for (int k = 0; k < DIM; ++k) {
    cm[k] = cell_coord(m[k], c.grid.lo[k], c.grid.cs);
    if (cm[k] < 1 || cm[k] > c.grid.n[k] - 2) return false;
  }
  constexpr int zr = DIM == 3 ? 1 : 0;
  for (int dz = -zr; dz <= zr; ++dz)
    for (int dy = -1; dy <= 1; ++dy) {
      const int base = ((cm[2] + dz) * A.ny + (cm[1] + dy)) * A.nx + cm[0];
      const int j0 = A.cs[base - 1], j3 = A.cs[base + 2];
      for (int j = j0 + lane; j < j3; j += L) {
        if (!is_real(A.tag[j])) continue;
        fn(j);
      }
    }
  (void)want_i_side;
  return true;
}

template <int DIM, int L>
__global__ __launch_bounds__(256) void k_adj_moment(AdjDev A, CorrAdjArgs c) {
  const int g = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int i = g / L, lane = g % L;
  if (i >= A.n) return;
  if (!is_real(A.tag[i])) {
    if (lane == 0)
      for (int k = 0; k < 6; ++k) A.cb[k][i] = 0.0;
    return;
  }
  const int64_t cap = A.cap;
  const double* xr[3] = {snap3(A.XR, cap, 0, 0), snap3(A.XR, cap, 0, 1), snap3(A.XR, cap, 0, 2)};
  double M[6] = {0, 0, 0, 0, 0, 0};
  auto acc = [&](const double r[3], double r2, double Vj) {
    double f, fp;
    kernel_f(sqrt(r2), A.inv_h, A.kf, f, fp);
    const double Vf = Vj * f;
    M[0] -= Vf * r[0] * r[0];
    M[1] -= Vf * r[0] * r[1];
    M[3] -= Vf * r[1] * r[1];
    if (DIM == 3) {
      M[2] -= Vf * r[0] * r[2];
      M[4] -= Vf * r[1] * r[2];
      M[5] -= Vf * r[2] * r[2];
    }
  };
  adj_neighbors<DIM, L>(A, xr, i, lane, [&](int j, const double r[3], double r2) {
    acc(r, r2, A.vol0[j]);
  });
  if (c.mirror) {
    const double xi[3] = {c.x[0][i], c.x[1][i], c.x[2][i]};
    for (int q = 0; q < c.nbuf; ++q) {
      const BufDev& b = c.bufs[q];
      double yi[3];
      to_local(b, xi[0], xi[1], xi[2], yi);
      if (!(yi[0] >= 0.0 && yi[0] < c.twoh)) continue;
      // no image within 2h beyond the buffer's transverse half-widths + 2h
      // (its particles keep their transverse coordinates in the mirror)
      const double reach = c.twoh * (1.0 + 1e-5);
      if (!(fabs(yi[1]) < b.hw[0] + reach) || (DIM == 3 && !(fabs(yi[2]) < b.hw[1] + reach)))
        continue;
      mirror_partners<DIM, L>(A, c, b, xi, lane, true, [&](int j) {
        double yj[3];
        const double xj0 = c.x[0][j], xj1 = c.x[1][j], xj2 = c.x[2][j];
        to_local(b, xj0, xj1, xj2, yj);
        if (!(yj[0] >= 0.0) || !contained(DIM, b, yj)) return;
        const double tj = 2.0 * yj[0];
        const double r[3] = {xi[0] - (xj0 - tj * b.frame[0]), xi[1] - (xj1 - tj * b.frame[1]),
                             DIM == 3 ? xi[2] - (xj2 - tj * b.frame[2]) : 0.0};
        const double r2 = DIM == 3 ? (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]
                                   : r[0] * r[0] + r[1] * r[1];
        if (r2 < A.rc2) acc(r, r2, A.vol0[j]);
      });
    }
  }
  team_sum_arr<L>(M);
  if (lane != 0) return;
  // reverse of the guarded inverse B = w A^-1 + (1 - w) I
  constexpr double theta = 0.25;
  double S[6];
  for (int k = 0; k < 6; ++k) S[k] = A.lB[k][i];
  if (DIM == 2) S[2] = S[4] = S[5] = 0.0;
  double inv[6], det, tr, d;
  if (DIM == 2) {
    tr = M[0] + M[3];
    det = M[0] * M[3] - M[1] * M[1];
    d = tr > 0.0 ? det / ((0.5 * tr) * (0.5 * tr)) : 0.0;
    inv[0] = M[3] / det; inv[1] = -M[1] / det; inv[3] = M[0] / det;
    inv[2] = inv[4] = inv[5] = 0.0;
  } else {
    const double c00 = M[3] * M[5] - M[4] * M[4];
    const double c01 = M[4] * M[2] - M[1] * M[5];
    const double c02 = M[1] * M[4] - M[3] * M[2];
    det = M[0] * c00 + M[1] * c01 + M[2] * c02;
    tr = M[0] + M[3] + M[5];
    const double t3 = tr / 3.0;
    d = tr > 0.0 ? det / (t3 * t3 * t3) : 0.0;
    inv[0] = c00 / det;
    inv[1] = c01 / det;
    inv[2] = c02 / det;
    inv[3] = (M[0] * M[5] - M[2] * M[2]) / det;
    inv[4] = (M[2] * M[1] - M[0] * M[4]) / det;
    inv[5] = (M[0] * M[3] - M[1] * M[1]) / det;
  }
  double Ab[6] = {0, 0, 0, 0, 0, 0};
  if (tr > 0.0 && d > 0.0) {
    const double w = d >= theta ? 1.0 : (d / theta) * (d / theta);
    double ISI[6];
    sym_sandwich<DIM>(inv, S, ISI);
    for (int k = 0; k < 6; ++k) Ab[k] = -w * ISI[k];
    if (d < theta) {
      const double id[6] = {1.0, 0.0, 0.0, 1.0, 0.0, DIM == 3 ? 1.0 : 0.0};
      double im[6];
      for (int k = 0; k < 6; ++k) im[k] = inv[k] - id[k];
      const double dLdw = sym_dot<DIM>(S, im);
      const double g = dLdw * 2.0 * d * d / (theta * theta);
      const double dimtr = (double)DIM / tr;
      for (int k = 0; k < 6; ++k) Ab[k] += g * (inv[k] - dimtr * id[k]);
    }
  }
  if (DIM == 2) Ab[2] = Ab[4] = Ab[5] = 0.0;
  for (int k = 0; k < 6; ++k) A.cb[k][i] = Ab[k];
}

// rT S r and S r for packed symmetric S.
template <int DIM>
__device__ __forceinline__ double quad(const double S[6], const double r[3], double Sr[3]) {
  symv_d<DIM>(S, r, Sr);
  return dot3(r, Sr);
}

template <int DIM, int L>
__global__ __launch_bounds__(256) void k_adj_correction(AdjDev A, CorrAdjArgs c) {
  const int g = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int i = g / L, lane = g % L;
  if (i >= A.n) return;
  if (!is_real(A.tag[i])) return;
  const int64_t cap = A.cap;
  const double* xr[3] = {snap3(A.XR, cap, 0, 0), snap3(A.XR, cap, 0, 1), snap3(A.XR, cap, 0, 2)};
  double Ci[6];
  for (int k = 0; k < 6; ++k) Ci[k] = A.cb[k][i];
  const double Vi = A.vol0[i];
  double acc[4] = {0, 0, 0, 0};   // lx, lV0
  adj_neighbors<DIM, L>(A, xr, i, lane, [&](int j, const double r[3], double r2) {
    const double rr = sqrt(r2);
    double f, fp;
    kernel_f(rr, A.inv_h, A.kf, f, fp);
    const double Vj = A.vol0[j];
    double Sr_i[3];
    const double qi = quad<DIM>(Ci, r, Sr_i);
    for (int k = 0; k < DIM; ++k) acc[k] -= Vj * (fp * r[k] / rr * qi + 2.0 * f * Sr_i[k]);
    if (tag_kind(A.tag[j]) == kWall) return;
    double Cj[6], Sr_j[3];
    for (int k = 0; k < 6; ++k) Cj[k] = A.cb[k][j];
    const double qj = quad<DIM>(Cj, r, Sr_j);
    for (int k = 0; k < DIM; ++k) acc[k] -= Vi * (fp * r[k] / rr * qj + 2.0 * f * Sr_j[k]);
    acc[3] += -f * qj;
  });
  if (c.mirror) {
    const double xk[3] = {c.x[0][i], c.x[1][i], c.x[2][i]};
    for (int q = 0; q < c.nbuf; ++q) {
      const BufDev& b = c.bufs[q];
      double yk[3];
      to_local(b, xk[0], xk[1], xk[2], yk);
      // i-side: images of partners j in A_i (none beyond the buffer's
      // transverse half-widths + 2h)
      const double reach = c.twoh * (1.0 + 1e-5);
      if (yk[0] >= 0.0 && yk[0] < c.twoh && fabs(yk[1]) < b.hw[0] + reach &&
          (DIM == 2 || fabs(yk[2]) < b.hw[1] + reach)) {
        mirror_partners<DIM, L>(A, c, b, xk, lane, true, [&](int j) {
          double yj[3];
          const double xj0 = c.x[0][j], xj1 = c.x[1][j], xj2 = c.x[2][j];
          to_local(b, xj0, xj1, xj2, yj);
          if (!(yj[0] >= 0.0) || !contained(DIM, b, yj)) return;
          const double tj = 2.0 * yj[0];
          const double r[3] = {xk[0] - (xj0 - tj * b.frame[0]), xk[1] - (xj1 - tj * b.frame[1]),
                               DIM == 3 ? xk[2] - (xj2 - tj * b.frame[2]) : 0.0};
          const double r2 = DIM == 3 ? (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]
                                     : r[0] * r[0] + r[1] * r[1];
          if (!(r2 < A.rc2)) return;
          const double rr = sqrt(r2);
          double f, fp;
          kernel_f(rr, A.inv_h, A.kf, f, fp);
          double Sr[3];
          const double qv = quad<DIM>(Ci, r, Sr);
          for (int k = 0; k < DIM; ++k)
            acc[k] -= A.vol0[j] * (fp * r[k] / rr * qv + 2.0 * f * Sr[k]);
        });
      }
      // j-side: this particle's image in the moments of the particles i
      // within 2h of the face (every i whose image search finds it)
      if (yk[0] >= 0.0 && contained(DIM, b, yk) && yk[0] < 1.25 * c.twoh) {
        const double tk = 2.0 * yk[0];
        const double xim[3] = {xk[0] - tk * b.frame[0], xk[1] - tk * b.frame[1],
                               xk[2] - tk * b.frame[2]};
        int cm[3] = {0, 0, 0};
        bool ok = true;
        for (int k = 0; k < DIM; ++k) {
          cm[k] = cell_coord(xim[k], c.grid.lo[k], c.grid.cs);
          if (cm[k] < 1 || cm[k] > c.grid.n[k] - 2) ok = false;
        }
        if (ok) {
          constexpr int zr = DIM == 3 ? 1 : 0;
          for (int dz = -zr; dz <= zr; ++dz)
            for (int dy = -1; dy <= 1; ++dy) {
              const int base = ((cm[2] + dz) * A.ny + (cm[1] + dy)) * A.nx + cm[0];
              const int j0 = A.cs[base - 1], j3 = A.cs[base + 2];
              for (int p = j0 + lane; p < j3; p += L) {
                if (!is_real(A.tag[p])) continue;
                const double xp0 = c.x[0][p], xp1 = c.x[1][p], xp2 = c.x[2][p];
                double yp[3];
                to_local(b, xp0, xp1, xp2, yp);
                if (!(yp[0] >= 0.0 && yp[0] < c.twoh)) continue;
                const double r[3] = {xp0 - (xk[0] - tk * b.frame[0]),
                                     xp1 - (xk[1] - tk * b.frame[1]),
                                     DIM == 3 ? xp2 - (xk[2] - tk * b.frame[2]) : 0.0};
                const double r2 = DIM == 3 ? (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]
                                           : r[0] * r[0] + r[1] * r[1];
                if (!(r2 < A.rc2)) continue;
                const double rr = sqrt(r2);
                double f, fp;
                kernel_f(rr, A.inv_h, A.kf, f, fp);
                double Cp[6], Sr[3];
                for (int k = 0; k < 6; ++k) Cp[k] = A.cb[k][p];
                const double qv = quad<DIM>(Cp, r, Sr);
                // dA_p/dx_k = -V_k [f' r_hat q + 2 f C r] (dr/dx_k = -H), H = I - 2 n n^T
                double gk[3];
                for (int k = 0; k < 3; ++k) gk[k] = Vi * (fp * r[k] / rr * qv + 2.0 * f * Sr[k]);
                const double ng = b.frame[0] * gk[0] + b.frame[1] * gk[1] + b.frame[2] * gk[2];
                for (int k = 0; k < DIM; ++k) acc[k] += gk[k] - 2.0 * b.frame[k] * ng;
                acc[3] += -f * qv;
              }
            }
        }
      }
    }
  }
  team_sum_arr<L>(acc);
  if (lane != 0) return;
  for (int k = 0; k < DIM; ++k) A.lx[k][i] += acc[k];
  A.lV0[i] += acc[3];
}

// Volumes V^0 = m / rho_0, then the cotangent of the start state by
// particle id; the copies created by the update get zero.
__global__ __launch_bounds__(256) void k_adj_finish(AdjDev A, double* lam, double mass) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  const uint32_t p = A.pid[i];
  if (p >= A.pid_cap) return;
  const int64_t pc = A.pid_cap;
  if (!is_real(A.tag[i])) {
    for (int k = 0; k < 8; ++k) lam[(int64_t)k * pc + p] = 0.0;
    return;
  }
  const double r0 = A.rho0[i];
  const double lr = A.lr[i] - mass / (r0 * r0) * A.lV0[i];
  for (int k = 0; k < 3; ++k) {
    lam[(int64_t)k * pc + p] = A.lx[k][i];
    lam[(int64_t)(3 + k) * pc + p] = A.lv[k][i];
  }
  lam[6 * pc + p] = lr;
  lam[7 * pc + p] = A.lDpre[i];
}

__global__ __launch_bounds__(256) void k_adj_zero_children(AdjDev A, double* lam) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  const int cp = A.child[i];
  if (cp < 0 || cp >= A.pid_cap) return;
  for (int k = 0; k < 8; ++k) lam[(int64_t)k * A.pid_cap + cp] = 0.0;
}

// grad[m] += sum_i abar[m][i] in a fixed order: per-block sums of all 16
// coefficients (tree in LDS), then one block per coefficient over the blocks.
__global__ __launch_bounds__(256) void k_adj_grad_part(int n, int64_t cap, const double* abar,
                                                       double* part) {
  __shared__ double sm[256];
  const int i = blockIdx.x * 256 + threadIdx.x;
  for (int m = 0; m < 16; ++m) {
    sm[threadIdx.x] = i < n ? abar[(int64_t)m * cap + i] : 0.0;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)m * gridDim.x + blockIdx.x] = sm[0];
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_adj_grad(int nb, const double* part, double* grad) {
  __shared__ double sm[256];
  const int m = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) s += part[(int64_t)m * nb + b];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) grad[m] += sm[0];
}

__global__ void k_zero_d(int64_t n, double* p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// ---------------------------------------------------------------------------
// Workspace layout.
// ---------------------------------------------------------------------------
struct AdjLayout {
  size_t total = 0;
  size_t take(size_t b) {
    size_t o = total;
    total += (b + 255) & ~size_t(255);
    return o;
  }
  size_t X, XR, V, RH, P, VOL, DD, rho0, vol0, tag, cot, abar, child, rec;
  // the step's cell build, neighbour list, correction and buffer update,
  // kept so that the reverse sweep does not depend on the context's state
  size_t pid, cell, cs, nbr, ncnt, stale, B, dec, inj;
  int ncot;
};

constexpr int kCot = 3 + 3 + 1 + 1 + 1 + 1 + 1 + 6 + 3 + 3 + 3 + 3 + 6 + 1;

AdjLayout adj_layout(const sph_ctx* c, int N) {
  AdjLayout L;
  const int64_t cap = c->cap;
  const size_t c8 = (size_t)cap * 8;
  L.X = L.take(c8 * 3 * (N + 1));
  L.XR = L.take(c8 * 3 * (N + 1));
  L.V = L.take(c8 * 3 * (N + 1));
  L.RH = L.take(c8 * (N + 1));
  L.P = L.take(c8 * N);
  L.VOL = L.take(c8 * N);
  L.DD = L.take(c8 * N);
  L.rho0 = L.take(c8);
  L.vol0 = L.take(c8);
  L.tag = L.take((size_t)cap * 4);
  L.cot = L.take(c8 * kCot);
  L.abar = L.take(c8 * 16);
  L.child = L.take((size_t)cap * 4);
  L.rec = L.take((size_t)cap * sizeof(V4<double>) *
                 (c->P.dim == 2 ? AdjRec<2>::nmax : AdjRec<3>::nmax));
  L.pid = L.take((size_t)cap * 4);
  L.cell = L.take((size_t)cap * 4);
  L.cs = L.take(((size_t)c->grid.ncell + 1) * 4);
  L.nbr = L.take((size_t)c->F.nbr_k * cap * 4);
  L.ncnt = L.take((size_t)cap * 4);
  L.stale = L.take(8);
  L.B = L.take(c8 * 6);
  L.dec = L.take((size_t)cap * 4);
  L.inj = L.take(((size_t)kMaxInject + 1) * 4);   // [0]: injections, then the slots
  L.ncot = kCot;
  return L;
}

AdjDev make_adj(sph_ctx* c, char* ws, const AdjLayout& L, int n, int64_t pid_cap) {
  AdjDev A;
  A.n = n;
  A.cap = c->cap;
  A.pid_cap = pid_cap;
  A.tag = (const uint32_t*)(ws + L.tag);
  A.pid = (const uint32_t*)(ws + L.pid);
  A.cell = (const int32_t*)(ws + L.cell);
  A.cs = (const int32_t*)(ws + L.cs);
  A.nx = c->grid.n[0];
  A.ny = c->grid.n[1];
  A.csz = c->P.cell_size;
  A.nbr = (const uint32_t*)(ws + L.nbr);   // used unless the kept stale words say so
  A.nk = c->F.nbr_k;
  A.ncnt = (const int32_t*)(ws + L.ncnt);
  A.stale = (const uint32_t*)(ws + L.stale);
  const double rc = 2.0 * c->P.h;
  A.rc2 = rc * rc;
  A.inv_h = 1.0 / c->P.h;
  const double h = c->P.h;
  const double alpha = c->P.dim == 2 ? 7.0 / (4.0 * M_PI * h * h) : 21.0 / (16.0 * M_PI * h * h * h);
  A.kf = -5.0 * alpha / (h * h);
  A.X = (double*)(ws + L.X);
  A.XR = (double*)(ws + L.XR);
  A.V = (double*)(ws + L.V);
  A.RH = (double*)(ws + L.RH);
  A.P = (double*)(ws + L.P);
  A.VOL = (double*)(ws + L.VOL);
  A.DD = (double*)(ws + L.DD);
  A.rho0 = (double*)(ws + L.rho0);
  A.vol0 = (double*)(ws + L.vol0);
  for (int k = 0; k < 6; ++k) A.B[k] = (const double*)(ws + L.B) + (int64_t)k * c->cap;
  double* cot = (double*)(ws + L.cot);
  int o = 0;
  auto nxt = [&]() { double* p = cot + (int64_t)o * c->cap; ++o; return p; };
  for (int k = 0; k < 3; ++k) A.lx[k] = nxt();
  for (int k = 0; k < 3; ++k) A.lv[k] = nxt();
  A.lr = nxt();
  A.lD = nxt();
  A.lDpre = nxt();
  A.lp = nxt();
  A.lV = nxt();
  for (int k = 0; k < 6; ++k) A.lB[k] = nxt();
  for (int k = 0; k < 3; ++k) A.la[k] = nxt();
  for (int k = 0; k < 3; ++k) A.qb[k] = nxt();
  for (int k = 0; k < 3; ++k) A.sb[k] = nxt();
  for (int k = 0; k < 3; ++k) A.ab[k] = nxt();
  for (int k = 0; k < 6; ++k) A.cb[k] = nxt();
  A.lV0 = nxt();
  A.abar = (double*)(ws + L.abar);
  A.child = (int32_t*)(ws + L.child);
  {
    const int nrec = c->P.dim == 2 ? AdjRec<2>::nmax : AdjRec<3>::nmax;
    V4<double>* r0 = (V4<double>*)(ws + L.rec);
    for (int w = 0; w < 5; ++w) A.rec[w] = w < nrec ? r0 + (int64_t)w * c->cap : nullptr;
  }
  A.flags = c->S.flags;
  return A;
}

#define ADJ_TEAM(L, ...)                                         \
  switch (L) {                                                   \
    case 1: { constexpr int TL = 1; __VA_ARGS__; } break;        \
    case 2: { constexpr int TL = 2; __VA_ARGS__; } break;        \
    case 4: { constexpr int TL = 4; __VA_ARGS__; } break;        \
    default: { constexpr int TL = 8; __VA_ARGS__; } break;       \
  }

int adj_team(const sph_ctx* c) {
  if (c->team_override > 0) return c->team_override;
  const int64_t n = c->n_total;
  if (n <= 120000) return 8;
  if (n <= 260000) return 4;
  if (n <= 450000) return 2;
  return 1;
}

// One snapshot entry: a source array, its FP64 destination, and whether the
// source is in the pair precision (float in an FP32-mixed context).
struct Snap {
  const void* src;
  double* dst;
  bool pair;
};

void snap_copy(sph_ctx* c, int n, std::initializer_list<Snap> lst) {
  CopyList cl;
  cl.k = 0;
  const bool f32 = c->P.precision != SPH_FP64;
  for (const Snap& e : lst) {
    cl.src[cl.k] = e.src;
    cl.dst[cl.k] = e.dst;
    cl.f32[cl.k] = e.pair && f32 ? 1 : 0;
    ++cl.k;
  }
  k_copy<<<nblk_a(n), 256, 0, c->stream>>>(n, cl);
}

template <int DIM>
hipError_t adjoint_reverse(sph_ctx* c, const AdjLayout& Lw, char* ws, const sph_objective_desc* obj,
                           const sph_adjoint_ctrl* ctl, int n, double* lam, double* grad) {
  const sph_params& P = c->P;
  AdjDev A = make_adj(c, ws, Lw, n, ctl->pid_cap);
  const int N = ctl->n_ac;
  const double dt = ctl->dt_adv / N;
  const double Vw = P.dim == 2 ? P.dp * P.dp : P.dp * P.dp * P.dp;
  const double mass = P.rho0 * Vw;
  const int nb = nblk_a(n);
  const int Lt = adj_team(c);
  hipStream_t st = c->stream;
  int control_q = -1;
  for (int q = 0; q < c->nbuf; ++q)
    if (c->bufs_h[q].id == obj->control_buffer) control_q = q;

  // children of the update
  k_fill_child<<<nb, 256, 0, st>>>(n, A.child);
  k_adj_children<<<(kMaxInject + 255) / 256, 256, 0, st>>>(
      A, (const int32_t*)(ws + Lw.inj), ctl->next_pid);
  // clear the cotangent accumulators
  k_zero_d<<<(int)(((int64_t)kCot * c->cap + 255) / 256), 256, 0, st>>>((int64_t)kCot * c->cap,
                                                                        A.lx[0]);
  k_zero_d<<<(int)((16 * c->cap + 255) / 256), 256, 0, st>>>(16 * c->cap, A.abar);

  PostArgs pa;
  pa.lam = lam;
  pa.dec = (const uint32_t*)(ws + Lw.dec);
  pa.bufs = c->S.bufs;
  pa.bidx = c->S.bidx;
  pa.control_q = control_q;
  pa.dim = P.dim;
  pa.seed = P.seed;
  pa.step_post = ctl->step + 1;
  pa.t_post = ctl->t + ctl->dt_adv;
  k_adj_post<<<nb, 256, 0, st>>>(A, pa, N);

  SeedArgs sa;
  sa.member = ctl->member_by_pid;
  sa.wq = ctl->w_flux;
  sa.wt = ctl->w_shear;
  for (int k = 0; k < 3; ++k) {
    sa.nrm[k] = obj->slab_normal[k];
    sa.e[k] = obj->shear_dir[k];
  }
  sa.w = obj->slab_width;
  sa.Lw = obj->wall_length;
  sa.m = mass;
  sa.mu = P.rho0 * P.nu_l;
  sa.Vw = Vw;
  ADJ_TEAM(Lt, k_adj_seed<DIM, TL><<<nblk_a((int64_t)n * TL), 256, 0, st>>>(A, sa, N));

  KickArgs ka;
  ka.bufs = c->S.bufs;
  ka.bidx = c->S.bidx;
  ka.control_q = control_q;
  ka.dim = P.dim;
  ka.mode = P.obc_mode;
  ka.seed = P.seed;
  ka.step = ctl->step;
  ka.t = ctl->t;
  ka.dt = dt;
  const double kappa = 1.0 / (2.0 * P.rho0 * P.c0);
  for (int s = N - 1; s >= 0; --s) {
    if (s == N - 1) k_adj_dprep<DIM><<<nb, 256, 0, st>>>(A, 1, 0.5 * dt, s);
    else k_adj_eos_dprep<DIM><<<nb, 256, 0, st>>>(A, s + 1, P.c0 * P.c0, mass, 0.5 * dt);
    ADJ_TEAM(Lt, k_adj_density<DIM, TL><<<nblk_a((int64_t)n * TL), 256, 0, st>>>(A, s, kappa));
    k_adj_kick<DIM><<<nb, 256, 0, st>>>(A, ka, s);
    switch (P.obc_mode) {
      case 1: ADJ_TEAM(Lt, k_adj_pressure<DIM, 1, TL><<<nblk_a((int64_t)n * TL), 256, 0, st>>>(A, ka, s)); break;
      case 2: ADJ_TEAM(Lt, k_adj_pressure<DIM, 2, TL><<<nblk_a((int64_t)n * TL), 256, 0, st>>>(A, ka, s)); break;
      case 3: ADJ_TEAM(Lt, k_adj_pressure<DIM, 3, TL><<<nblk_a((int64_t)n * TL), 256, 0, st>>>(A, ka, s)); break;
      default: ADJ_TEAM(Lt, k_adj_pressure<DIM, 4, TL><<<nblk_a((int64_t)n * TL), 256, 0, st>>>(A, ka, s)); break;
    }
  }
  k_adj_eos<<<nb, 256, 0, st>>>(A, 0, P.c0 * P.c0, mass);
  k_adj_vprep<<<nb, 256, 0, st>>>(A, 2.0 * P.rho0 * P.nu_l, 0.5 * dt);
  ADJ_TEAM(Lt, k_adj_viscous<DIM, TL><<<nblk_a((int64_t)n * TL), 256, 0, st>>>(A));
  if (P.obc_mode >= 2) {
    CorrAdjArgs ca;
    const double* X0 = A.X;
    for (int k = 0; k < 3; ++k) ca.x[k] = X0 + (int64_t)k * c->cap;
    ca.bufs = c->S.bufs;
    ca.nbuf = c->nbuf;
    ca.mirror = P.obc_mode >= 3 ? 1 : 0;
    ca.twoh = 2.0 * P.h;
    ca.grid = c->grid;
    ADJ_TEAM(Lt, k_adj_moment<DIM, TL><<<nblk_a((int64_t)n * TL), 256, 0, st>>>(A, ca));
    ADJ_TEAM(Lt, k_adj_correction<DIM, TL><<<nblk_a((int64_t)n * TL), 256, 0, st>>>(A, ca));
  }
  k_adj_finish<<<nb, 256, 0, st>>>(A, lam, mass);
  k_adj_zero_children<<<nb, 256, 0, st>>>(A, lam);
  // per-block partials of the gradient reuse the (consumed) sub-step
  // density snapshots: 16 x nb doubles
  double* gpart = A.DD;
  k_adj_grad_part<<<nb, 256, 0, st>>>(n, c->cap, A.abar, gpart);
  k_adj_grad<<<16, 256, 0, st>>>(nb, gpart, grad);
  return hipGetLastError();
}

}  // namespace

size_t adjoint_ws_bytes(const sph_ctx* c, int max_nac) {
  if (c->P.turbulence || c->P.tvf_alpha != 0.0 || max_nac < 1) return 0;
  return adj_layout(c, max_nac).total;
}

hipError_t launch_objective(sph_ctx* c, const sph_objective_desc* obj, const uint8_t* member_in,
                            uint8_t* member_out, int64_t pid_cap, double* J) {
  const sph_params& P = c->P;
  const int64_t n = c->n_total;
  ObjArgs a;
  for (int k = 0; k < 3; ++k) {
    a.o[k] = obj->slab_origin[k];
    a.nrm[k] = obj->slab_normal[k];
    a.e[k] = obj->shear_dir[k];
    a.x[k] = c->F.x[k].live();
  }
  a.w = obj->slab_width;
  a.Lw = obj->wall_length;
  a.Vw = P.dim == 2 ? P.dp * P.dp : P.dp * P.dp * P.dp;
  a.m = P.rho0 * a.Vw;
  a.mu = P.rho0 * P.nu_l;
  a.rho = c->F.rho.live();
  a.member_in = member_in;
  a.member_out = member_out;
  a.pid_cap = pid_cap;
  a.part = c->S.red + 4;
  const int nb = nblk_a(n);
  if (member_out)
    k_fill_u8<<<(int)((pid_cap + 255) / 256), 256, 0, c->stream>>>(pid_cap, member_out);
  if (P.precision == SPH_FP64) {
    PairCtx<double> pc = make_pc<double>(c, c->F.xr, c->F.x[0].cur);
    pc.pairs = nullptr;
    Consts<double> C = make_consts<double>(c);
    const double* v[3] = {tp<double>(c->F.v[0].live()), tp<double>(c->F.v[1].live()),
                          tp<double>(c->F.v[2].live())};
    if (P.dim == 2)
      k_objective<double, 2><<<nb, 256, 0, c->stream>>>((int)n, pc, C, v[0], v[1], v[2], c->F.pid.live(), a);
    else
      k_objective<double, 3><<<nb, 256, 0, c->stream>>>((int)n, pc, C, v[0], v[1], v[2], c->F.pid.live(), a);
  } else {
    PairCtx<float> pc = make_pc<float>(c, c->F.xr, c->F.x[0].cur);
    pc.pairs = nullptr;
    Consts<float> C = make_consts<float>(c);
    const float* v[3] = {tp<float>(c->F.v[0].live()), tp<float>(c->F.v[1].live()),
                         tp<float>(c->F.v[2].live())};
    if (P.dim == 2)
      k_objective<float, 2><<<nb, 256, 0, c->stream>>>((int)n, pc, C, v[0], v[1], v[2], c->F.pid.live(), a);
    else
      k_objective<float, 3><<<nb, 256, 0, c->stream>>>((int)n, pc, C, v[0], v[1], v[2], c->F.pid.live(), a);
  }
  k_objective_final<<<1, 256, 0, c->stream>>>(nb, a.part, a.Lw, J);
  return hipGetLastError();
}

// Snapshot hooks of the replayed forward step (FP64 context).
hipError_t adjoint_snap_start(sph_ctx* c, char* ws, int N) {
  AdjLayout L = adj_layout(c, N);
  const int n = (int)c->n_total;
  const int64_t cap = c->cap;
  double* X = (double*)(ws + L.X);
  double* XR = (double*)(ws + L.XR);
  double* V = (double*)(ws + L.V);
  Fields& F = c->F;
  snap_copy(c, n, {{F.x[0].live(), X, false}, {F.x[1].live(), X + cap, false},
                   {F.x[2].live(), X + 2 * cap, false}, {F.xr[0].live(), XR, true},
                   {F.xr[1].live(), XR + cap, true}, {F.xr[2].live(), XR + 2 * cap, true},
                   {F.v[0].live(), V, true}, {F.v[1].live(), V + cap, true},
                   {F.v[2].live(), V + 2 * cap, true}, {F.rho.live(), (double*)(ws + L.rho0), false}});
  snap_copy(c, n, {{F.vol.live(), (double*)(ws + L.vol0), true}});
  k_copy_u32<<<nblk_a(n), 256, 0, c->stream>>>(n, F.tag.live(), (uint32_t*)(ws + L.tag));
  return hipGetLastError();
}

hipError_t adjoint_snap_advection(sph_ctx* c, char* ws, int N) {
  AdjLayout L = adj_layout(c, N);
  const int n = (int)c->n_total;
  Fields& F = c->F;
  snap_copy(c, n, {{F.rho.live(), (double*)(ws + L.RH), false},
                   {F.p.live(), (double*)(ws + L.P), true},
                   {F.vol.live(), (double*)(ws + L.VOL), true}});
  return hipGetLastError();
}

hipError_t adjoint_snap_pressure(sph_ctx* c, char* ws, int N, int s) {
  AdjLayout L = adj_layout(c, N);
  const int n = (int)c->n_total;
  const int64_t cap = c->cap;
  const int64_t o = (int64_t)(s + 1) * 3 * cap;
  double* X = (double*)(ws + L.X) + o;
  double* XR = (double*)(ws + L.XR) + o;
  double* V = (double*)(ws + L.V) + o;
  Fields& F = c->F;
  snap_copy(c, n, {{F.x[0].live(), X, false}, {F.x[1].live(), X + cap, false},
                   {F.x[2].live(), X + 2 * cap, false}, {F.xr[0].live(), XR, true},
                   {F.xr[1].live(), XR + cap, true}, {F.xr[2].live(), XR + 2 * cap, true},
                   {F.v[0].live(), V, true}, {F.v[1].live(), V + cap, true},
                   {F.v[2].live(), V + 2 * cap, true}});
  return hipGetLastError();
}

hipError_t adjoint_snap_density(sph_ctx* c, char* ws, int N, int s) {
  AdjLayout L = adj_layout(c, N);
  const int n = (int)c->n_total;
  const int64_t cap = c->cap;
  Fields& F = c->F;
  double* DD = (double*)(ws + L.DD) + (int64_t)s * cap;
  double* RH = (double*)(ws + L.RH) + (int64_t)(s + 1) * cap;
  if (s < N - 1)
    snap_copy(c, n, {{F.drho.live(), DD, true}, {F.rho.live(), RH, false},
                     {F.p.live(), (double*)(ws + L.P) + (int64_t)(s + 1) * cap, true},
                     {F.vol.live(), (double*)(ws + L.VOL) + (int64_t)(s + 1) * cap, true}});
  else
    snap_copy(c, n, {{F.drho.live(), DD, true}, {F.rho.live(), RH, false}});
  return hipGetLastError();
}

// After the step's buffer update: the build, list, correction and update
// data of the step into the workspace (the list only while it was built;
// otherwise the kept stale words send the reverse passes to the stencil).
hipError_t adjoint_keep_step(sph_ctx* c, char* ws, int N, int n_step) {
  AdjLayout L = adj_layout(c, N);
  hipStream_t st = c->stream;
  const int64_t cap = c->cap;
  const int n_after = (int)c->n_total;
  hipError_t e = hipMemcpyAsync(ws + L.pid, c->F.pid.live(), (size_t)n_after * 4,
                                hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ws + L.cell, c->F.cell, (size_t)n_step * 4, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ws + L.cs, c->S.cell_start, ((size_t)c->grid.ncell + 1) * 4,
                       hipMemcpyDeviceToDevice, st);
  const bool list = c->use_nbr && c->nbr_valid;
  if (e == hipSuccess && list && n_step > 0) {
    // rows of chunks (nbr_index): C entries of every particle per row
    const size_t C = c->P.dim == 3 ? nbr_chunk<3>() : nbr_chunk<2>();
    e = hipMemcpy2DAsync(ws + L.nbr, (size_t)cap * 4 * C, c->F.nbr, (size_t)cap * 4 * C,
                         (size_t)n_step * 4 * C, (size_t)c->F.nbr_k / C,
                         hipMemcpyDeviceToDevice, st);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(ws + L.ncnt, c->F.ncnt, (size_t)n_step * 4, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) {
    if (list) e = hipMemcpyAsync(ws + L.stale, c->S.stale, 8, hipMemcpyDeviceToDevice, st);
    else e = hipMemsetAsync(ws + L.stale, 0xFF, 8, st);
  }
  if (e == hipSuccess && n_step > 0) {
    double* B = (double*)(ws + L.B);
    snap_copy(c, n_step, {{c->F.B[0], B, true}, {c->F.B[1], B + cap, true},
                          {c->F.B[2], B + 2 * cap, true}, {c->F.B[3], B + 3 * cap, true},
                          {c->F.B[4], B + 4 * cap, true}, {c->F.B[5], B + 5 * cap, true}});
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(ws + L.dec, c->S.dec, (size_t)n_step * 4, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ws + L.inj, c->S.counters + 1024, 4, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ws + L.inj + 4, c->S.inj_idx, (size_t)kMaxInject * 4,
                       hipMemcpyDeviceToDevice, st);
  return e;
}

hipError_t adjoint_reverse_launch(sph_ctx* c, char* ws, const sph_objective_desc* obj,
                                  const sph_adjoint_ctrl* ctl, int n, double* lam, double* grad) {
  AdjLayout L = adj_layout(c, ctl->n_ac);
  return c->P.dim == 2 ? adjoint_reverse<2>(c, L, ws, obj, ctl, n, lam, grad)
                       : adjoint_reverse<3>(c, L, ws, obj, ctl, n, lam, grad);
}

}  // namespace sphx
