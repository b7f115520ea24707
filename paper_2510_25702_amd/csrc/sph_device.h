// Device-side building blocks of the gfx950 SPH pipeline: constants,
// kernel function, buffer geometry, counter-based random numbers and
// wave64 scans.  Shared by the kernel translation units of this library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sphx {

constexpr int kMaxBuf = 32;
constexpr int kMaxInject = 4096;
constexpr int kWave = 64;
constexpr int kNbrMax2 = 64;            // neighbour-list entries per particle (2D)
constexpr int kNbrMax3 = 256;           // (3D)
// list entry = j | (dx + 1) << 26 | (dy + 1) << 28 | (dz + 1) << 30, with
// (dx, dy, dz) the cell of j relative to the cell of i
constexpr int kNbrIdxBits = 26;
constexpr int kNbrNoList = 0x7FFFFFFF;  // list count of a particle whose list overflowed
constexpr uint32_t kNbrIdxMask = (1u << kNbrIdxBits) - 1u;
// Entry k of particle i in the per-step neighbour list: chunks of C
// consecutive entries of one particle, chunk c of every particle in one row
// of `stride` chunks.  3D lists (about 170 entries) take C = 4 (16 bytes): a
// particle's appends stay within a few lines and a team reads whole chunks
// (the 3.75M-particle mixer's list build 6.50 -> 5.22 ms).  2D lists (about
// 36 entries) keep C = 1, one row per entry: there the 16-byte chunks made
// the passes at 2.56M particles 10-15 % slower and gained nothing at 57.6k.
template <int DIM>
constexpr int nbr_chunk() {
  return DIM == 3 ? 4 : 1;
}
template <int DIM>
__host__ __device__ inline int64_t nbr_index(int k, int i, int64_t stride) {
  constexpr uint32_t C = nbr_chunk<DIM>();
  // k, i >= 0 and stride < 2^26: unsigned shifts and one 32 x 32 -> 64 product
  const uint32_t ku = (uint32_t)k;
  return (int64_t)(((uint64_t)(ku / C) * (uint32_t)stride + (uint32_t)i) * C + ku % C);
}
constexpr int kPairShards = 64;        // pair counters, one per 128-byte line
constexpr int kPairShardStride = 16;    // long longs between two counters

enum : uint32_t { kFluid = 0, kBuffer = 1, kWall = 2, kDead = 3 };
enum : uint32_t { kVelExtrapolate = 0, kVelPrescribed = 1 };
enum : uint32_t { kPNone = 0, kPPrescribed = 1, kPExtrapolate = 2 };
enum : uint32_t { kTurbZeroGradient = 0, kTurbFreestream = 1 };
enum : uint32_t { kProfUniform = 0, kProfParabolic = 1, kProfSine = 2 };
enum : uint32_t { kDecNone = 0, kDecRelabel = 1, kDecInject = 2, kDecDelete = 3,
                  kDecRevert = 4, kDecRevertRelabel = 5 };

// error flags raised by kernels (device word, read at synchronisation points)
enum : uint32_t { kFlagOutOfGrid = 1u, kFlagSkin = 2u, kFlagNonFinite = 4u,
                  kFlagInjectOverflow = 8u, kFlagCapacity = 16u,
                  kFlagCountMismatch = 32u };

__host__ __device__ inline uint32_t tag_kind(uint32_t t) { return t & 3u; }
__host__ __device__ inline uint32_t tag_bid(uint32_t t) { return (t >> 8) & 0xFFu; }
__host__ __device__ inline bool is_real(uint32_t t) { return (t & 3u) <= kBuffer; }

// Buffer table entry in device memory (copied from sph_buffer_desc, plus
// derived values computed once on the host).
struct BufDev {
  int32_t id, vel_mode, p_mode, turb_mode, profile, n_coef;
  double origin[3];
  double frame[9];
  double length, hw[2], fringe;
  double gen;          // length + fringe: particle-generation line
  double p_ob, k_bc, eps_bc, u0, noise_amp, ramp_time;
  double rho_bc;       // density of Eq. (eos) at p_ob
  double coef[16];
  int32_t clo[3], chi[3];   // local cell-linked-list box (cell coordinates)
};

struct GridDev {
  double lo[3];
  double cs;
  int32_t n[3];
  int32_t ncell;
};

// Scalars of the problem, in FP64 and in the pair precision T.
template <typename T>
struct Consts {
  int32_t dim, turbulence, obc_mode, nbuf;
  GridDev grid;
  double h, rc2, dp, Vw, mass, rho0, c0, nu_l, eta, g[3];
  double C1, C2, Cmu, sigma_k, sigma_eps, k_floor, eps_floor;
  double skin;          // allowed distance of a particle outside its build cell
  uint64_t seed;
  T h_t, rc2_t, cs_t, inv_h_t, kf_t;  // kf = -5 alpha / h^2 (dW/dr / r prefactor)
  double inv_h_d, kf_d;               // the same in FP64
  T rho0_t, c0_t, eta_t, inv_2rc0_t, mu_R_t;   // mu_R_t = rho0 h / 2
};

// ---------------------------------------------------------------------------
// Wendland C2 kernel: W = alpha (1 - q/2)^4 (2q + 1), q = r / h < 2;
// (dW/dr) / r = -5 alpha (1 - q/2)^3 / h^2.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T dw_over_r(T r, T inv_h, T kf) {
  T t = T(1) - T(0.5) * r * inv_h;
  return kf * t * t * t;
}

// Pair distance |r| from r^2 in the pair passes.  FP32: the hardware square
// root, within one ulp (the correctly rounded library sequence adds about
// fifteen instructions per candidate, executed by the whole wavefront, far
// below the FP32-mixed pair terms' own rounding).  FP64: the library one.
__device__ __forceinline__ float pair_dist(float r2) { return __builtin_amdgcn_sqrtf(r2); }
__device__ __forceinline__ double pair_dist(double r2) { return sqrt(r2); }

// ---------------------------------------------------------------------------
// Buffer geometry in FP64 without contraction (bit-reproducible predicates).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double dmul(double a, double b) { return __dmul_rn(a, b); }
__device__ __forceinline__ double dadd(double a, double b) { return __dadd_rn(a, b); }
__device__ __forceinline__ double dsub(double a, double b) { return __dsub_rn(a, b); }

__device__ __forceinline__ void to_local(const BufDev& b, double x0, double x1, double x2,
                                         double y[3]) {
  double d0 = dsub(x0, b.origin[0]), d1 = dsub(x1, b.origin[1]), d2 = dsub(x2, b.origin[2]);
#pragma unroll
  for (int k = 0; k < 3; ++k)
    y[k] = dadd(dadd(dmul(b.frame[3 * k], d0), dmul(b.frame[3 * k + 1], d1)),
                dmul(b.frame[3 * k + 2], d2));
}

__device__ __forceinline__ bool contained(int dim, const BufDev& b, const double y[3]) {
  if (fabs(y[1]) > b.hw[0]) return false;
  if (dim == 3 && fabs(y[2]) > b.hw[1]) return false;
  return true;
}

__device__ __forceinline__ int cell_coord(double x, double lo, double cs) {
  return (int)floor(__ddiv_rn(dsub(x, lo), cs));
}

// Centre of cell c along one axis: the origin of the cell-relative positions
// (|x - centre| <= cs / 2 + skin, one bit more of FP32 precision than
// positions relative to the cell's corner).
__host__ __device__ inline double cell_centre(double lo, int c, double cs) {
  return lo + ((double)c + 0.5) * cs;
}

// Quarter of its cell along x of a cell-relative position (0..3, from the
// low face): the cell build orders each cell by it, so that a stencil scan
// can leave out the quarters of the neighbouring cells that lie beyond its
// radius.
__device__ __forceinline__ int x_quarter(double rel, double cs) {
  const int q = (int)floor((rel + 0.5 * cs) * (4.0 / cs));
  return q < 0 ? 0 : (q > 3 ? 3 : q);
}

// ---------------------------------------------------------------------------
// SplitMix64 (Steele, Lea & Flood 2014) and the counter-based uniform number
// u = 2 (z >> 11) 2^-53 - 1, z = mix(mix(mix(seed) ^ pid) ^ (step << 2 | c)).
// ---------------------------------------------------------------------------
__host__ __device__ inline uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__host__ __device__ inline double counter_uniform(uint64_t seed, uint32_t pid, int64_t step,
                                                  uint32_t comp) {
  uint64_t z = splitmix64(seed);
  z = splitmix64(z ^ (uint64_t)pid);
  z = splitmix64(z ^ (((uint64_t)step << 2) | (uint64_t)comp));
  return (double)(z >> 11) * 0x1.0p-53 * 2.0 - 1.0;
}

// Start-up ramp of a buffer's prescribed values: 0.5 (1 - cos(pi t / T)).
__device__ __forceinline__ double buffer_ramp(const BufDev& b, double t) {
  if (b.ramp_time > 0.0 && t < b.ramp_time) return 0.5 * (1.0 - cos(M_PI * t / b.ramp_time));
  return 1.0;
}

// Density of Eq. (eos) at pressure p (laminar).
__device__ __forceinline__ double rho_of_p(double rho0, double c0, double p) {
  const double den = __dmul_rn(__dmul_rn(rho0, c0), c0);
  return __dmul_rn(rho0, __dadd_rn(__ddiv_rn(p, den), 1.0));
}

// Prescribed speed along n_b of a buffer (Table 3 velocity inlets):
// uniform / parabolic / parabola + sine series, times the optional noise and
// start-up ramp.  y = local coordinates of the particle.
__device__ inline double profile_speed(int dim, const BufDev& b, const double y[3],
                                       uint64_t seed, uint32_t pid, int64_t step, double t) {
  double s = (y[1] + b.hw[0]) / (2.0 * b.hw[0]);
  double u;
  if (b.profile == kProfParabolic) {
    u = 4.0 * b.u0 * s * (1.0 - s);
    if (dim == 3) {
      double tt = (y[2] + b.hw[1]) / (2.0 * b.hw[1]);
      u *= 4.0 * tt * (1.0 - tt);
    }
  } else if (b.profile == kProfSine) {
    u = 4.0 * b.u0 * s * (1.0 - s);
    for (int m = 1; m <= b.n_coef; ++m) u += b.coef[m - 1] * sin((double)m * M_PI * s);
  } else {
    u = b.u0;
  }
  if (b.noise_amp != 0.0) u *= 1.0 + b.noise_amp * counter_uniform(seed, pid, step, 0);
  return u * buffer_ramp(b, t);
}

// ---------------------------------------------------------------------------
// XCD-aware block order.  Workgroups of a launch are dealt to the 8 XCDs in
// turn (block b runs on XCD b mod 8), each XCD with its own L2.  Mapping the
// hardware block id to a logical one so that each XCD receives one
// contiguous range of logical blocks keeps neighbouring cells (whose
// particles re-read each other's fields) in the same L2.  A bijection on
// [0, nblocks).
// ---------------------------------------------------------------------------
constexpr int kXcds = 8;

__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int x = b % kXcds, q = b / kXcds;
  const int per = nb / kXcds, rem = nb % kXcds;
  return x < rem ? x * (per + 1) + q : rem * (per + 1) + (x - rem) * per + q;
}

// ---------------------------------------------------------------------------
// wave64 / block scans
// ---------------------------------------------------------------------------
// Cell id of slot i (FP64, floor((x - lo) / cs), IEEE division; -1 for a
// particle tagged dead or a slot at or beyond n) and its slot inside the
// cell.  The particles arrive (mostly) in the previous build's cell order,
// so each run of equal ids along the wavefront takes its slots with one
// atomic on its cell count.  Every lane of the wavefront must call this
// with consecutive slots.
template <int DIM>
__device__ __forceinline__ void cell_key_slot(int i, int n, const double* __restrict__ x0,
                                              const double* __restrict__ x1,
                                              const double* __restrict__ x2,
                                              const uint32_t* __restrict__ tag, const GridDev& g,
                                              int32_t* __restrict__ key,
                                              int32_t* __restrict__ slot, int32_t* count,
                                              uint32_t* __restrict__ flags) {
  const int lane = threadIdx.x & (kWave - 1);
  int id = -1;
  if (i < n && tag_kind(tag[i]) != kDead) {
    const double* xs[3] = {x0, x1, x2};
    int c[3] = {0, 0, 0};
    bool bad = false;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      double q = floor(__ddiv_rn(__dsub_rn(xs[k][i], g.lo[k]), g.cs));
      if (!(q >= 1.0 && q <= (double)(g.n[k] - 2))) {
        bad = true;
        q = (q >= 1.0) ? (double)(g.n[k] - 2) : 1.0;   // also catches NaN
      }
      c[k] = (int)q;
    }
    if (bad) atomicOr(flags, kFlagOutOfGrid);
    id = (c[2] * g.n[1] + c[1]) * g.n[0] + c[0];
  }
  // runs of equal keys: the head lane reserves the run's slots
  const int prev = __builtin_amdgcn_update_dpp(0, id, 0x138, 0xF, 0xF, false);   // wave_shr:1
  const bool head = lane == 0 || prev != id;
  const uint64_t heads = __ballot(head);
  const uint64_t upto = lane == kWave - 1 ? ~0ull : ((2ull << lane) - 1ull);
  const int h = 63 - __clzll(heads & upto);
  const uint64_t after = heads & ~upto;
  const int next = after ? __ffsll((unsigned long long)after) - 1 : kWave;
  int base = 0;
  if (head && id >= 0) base = atomicAdd(&count[id], next - lane);
  base = __shfl(base, h, kWave);
  if (i < n) {
    key[i] = id;
    if (id >= 0) slot[i] = base + (lane - h);
  }
}

// Inclusive scan over the 64 lanes with DPP register moves (no LDS): a
// Hillis-Steele scan inside each row of 16 lanes (row_shr 1, 2, 4, 8; a lane
// with no source reads 0), then lane 15 of each row added to the next row
// (rows 1 and 3) and lane 31 added to rows 2 and 3.
__device__ __forceinline__ int wave_incl_scan(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, false);   // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, false);   // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, false);   // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, false);   // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);   // row_bcast:15
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);   // row_bcast:31
  return v;
}

// Exclusive scan over the block; `sm` holds >= blockDim.x / 64 ints.
__device__ __forceinline__ int block_excl_scan(int v, int* sm, int* total) {
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  int inc = wave_incl_scan(v);
  if (lane == kWave - 1) sm[wid] = inc;
  __syncthreads();
  if (wid == 0) {
    int s = lane < nw ? sm[lane] : 0;
    int si = wave_incl_scan(s);
    if (lane < nw) sm[lane] = si - s;
    if (lane == nw - 1) sm[nw] = si;
  }
  __syncthreads();
  int r = inc - v + sm[wid];
  if (total) *total = sm[nw];
  __syncthreads();
  return r;
}

// Lane l's view of lane l ^ O by DPP register moves (no LDS): quad
// permutations for O = 1, 2; for O = 4 the row shifted by 4 either way,
// chosen by lane bit 2; for O = 8 the 16-lane row rotated by 8.
template <int CTRL>
__device__ __forceinline__ int dpp_move(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int O>
__device__ __forceinline__ int lane_xor_i32(int v) {
  if constexpr (O == 1) return dpp_move<0xB1>(v);            // quad_perm [1,0,3,2]
  else if constexpr (O == 2) return dpp_move<0x4E>(v);       // quad_perm [2,3,0,1]
  else if constexpr (O == 4) {
    const int up = dpp_move<0x104>(v), down = dpp_move<0x114>(v);   // row_shl:4, row_shr:4
    return (threadIdx.x & 4) ? down : up;
  } else if constexpr (O == 8) return dpp_move<0x128>(v);     // row_ror:8
  else return __shfl_xor(v, O, kWave);
}
template <int O, typename T>
__device__ __forceinline__ T lane_xor(T v) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, lane_xor_i32<O>(__builtin_bit_cast(int, v)));
  } else {
    static_assert(sizeof(T) == 8, "32- or 64-bit values");
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)lane_xor_i32<O>((int)(uint32_t)u);
    const uint32_t hi = (uint32_t)lane_xor_i32<O>((int)(uint32_t)(u >> 32));
    return __builtin_bit_cast(T, ((uint64_t)hi << 32) | (uint64_t)lo);
  }
}

// lane_xor with the distance known after unrolling (a power of two < 64)
template <typename T>
__device__ __forceinline__ T lane_xor_by(T v, int o) {
  switch (o) {
    case 1: return lane_xor<1>(v);
    case 2: return lane_xor<2>(v);
    case 4: return lane_xor<4>(v);
    case 8: return lane_xor<8>(v);
    case 16: return lane_xor<16>(v);
    default: return lane_xor<32>(v);
  }
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    T t = __shfl_xor(v, o, kWave);
    v = v > t ? v : t;
  }
  return v;
}

__device__ __forceinline__ long long wave_sum_ll(long long v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Four pair-precision values, loaded and stored as one 16-byte (float) or
// two 16-byte (double) vector accesses: the j-side records of the
// neighbour passes.
template <typename T>
struct alignas(4 * sizeof(T)) V4 {
  T a, b, c, d;
};

// Record of particle j for the advection pass, written by the cell build:
// position, velocity, V (negative for a wall) and the RANS fields.
// 2D: {x0, x1, v0, v1} {Vw, nut, k, eps};
// 3D: {x0, x1, x2, v0} {v1, v2, Vw, nut} {k, eps, 0, 0} (the third only with RANS).
template <typename T, int DIM>
__device__ __forceinline__ void write_arec(V4<T>* const* ar, int i, const T x[3], const T v[3],
                                           T volw, T nut, T k, T eps, bool turb) {
  if (DIM == 2) {
    ar[0][i] = V4<T>{x[0], x[1], v[0], v[1]};
    ar[1][i] = V4<T>{volw, nut, k, eps};
  } else {
    ar[0][i] = V4<T>{x[0], x[1], x[2], v[0]};
    ar[1][i] = V4<T>{v[1], v[2], volw, nut};
    if (turb) ar[2][i] = V4<T>{k, eps, T(0), T(0)};
  }
}

}  // namespace sphx
