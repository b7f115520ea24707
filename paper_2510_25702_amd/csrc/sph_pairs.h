// Neighbour-pass building blocks shared by the forward passes (k_pairs.hip)
// and their adjoints (k_adjoint.hip): the cell-stencil neighbour loop and
// the list walks over packed records with teams of lanes per particle, the
// list build of the correction, team reductions, the sharded pair counter,
// small symmetric-matrix helpers, the equation of state and the guarded
// inverse of the correction moment.
#pragma once

#include <type_traits>

#include "sph_ctx.h"

namespace sphx {

template <typename T>
inline T* tp(void* p) { return static_cast<T*>(p); }

template <typename T>
struct PairCtx {
  const T* xr[3];
  const T* vol;
  const uint32_t* tag;
  const int32_t* cell;
  const int32_t* cs;    // cell_start
  int nx, ny;
  T csz, rc2, inv_h, kf;
  long long* pairs;   // directed pairs counter (NULL: not counted)
  const uint32_t* nbr;  // per-step neighbour list (NULL: scan the cell stencil)
  const int32_t* ncnt;
  int64_t nstride;
  int nk;               // rows of the list (every one allocated)
  const uint32_t* stale;  // non-zero: the list no longer covers the positions
};

// Launch of a neighbour pass (256-thread workgroups on the context stream);
// under profiling the launch records the section's events itself.
template <typename... KArgs, typename... Args>
inline void launch_pass(sph_ctx* c, void (*k)(KArgs...), int64_t grid, Args... args) {
  hipEvent_t a = c->prof.ext_a, b = c->prof.ext_b;
  c->prof.ext_a = c->prof.ext_b = nullptr;
  if (a) hipExtLaunchKernelGGL(k, dim3((unsigned)grid), dim3(256), 0, c->stream, a, b, 0, args...);
  else hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(256), 0, c->stream, args...);
}

// Sum over the L lanes of a team (butterfly: the same order in every run).
template <int L, typename T>
__device__ __forceinline__ T team_sum(T v) {
  if constexpr (L >= 2) {
    v += lane_xor<L / 2>(v);
    return team_sum<L / 2>(v);
  }
  return v;
}

// Directed-pair counter: one atomic per block, spread over kPairShards
// counters 128 bytes apart, so the passes do not serialise on one address.
// Every thread of the block must reach this call.
__device__ __forceinline__ void count_pairs(long long* ctr, long long m) {
  if (!ctr) return;
  __shared__ long long part[16];
  // a wavefront's pairs fit in 32 bits: its inclusive scan ends in lane 63
  const int tot = wave_incl_scan((int)m);
  const int nw = blockDim.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == kWave - 1) part[threadIdx.x / kWave] = tot;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long s = 0;
    for (int w = 0; w < nw; ++w) s += part[w];
    if (s)
      atomicAdd(reinterpret_cast<unsigned long long*>(ctr + (blockIdx.x & (kPairShards - 1)) *
                                                               kPairShardStride),
                (unsigned long long)s);
  }
}

// Visit every j != i with |r_ij|^2 < (2h)^2 among the particles of the
// 3^DIM build cells around i's cell; r = x_i - x_j from cell-relative
// positions: r = (xr_i - xr_j) - (cell_j - cell_i) * cs.
// A team of L consecutive lanes shares particle i: lane l visits the
// candidates l, l + L, l + 2L, ... .  The candidates are taken kUnroll at a
// time: their positions are loaded together before any is tested, so that
// the loads of one batch are in flight at once.
// With a neighbour list (built with B after the cell build, radius = cell
// size) the candidates are its entries (in stencil order, shared among the
// lanes as list_vec states): the same pairs as the stencil scan, summed per
// lane in another grouping.  The list covers every
// pair within 2h while no particle has moved more than (cell size - 2h) / 2
// since it was built; the pressure pass flags the step's list as outgrown
// otherwise, and the later passes of the step scan the stencil instead.
#ifndef SPHX_UNROLL
#define SPHX_UNROLL 2
#endif
constexpr int kUnroll = SPHX_UNROLL;

// List entry of candidate j in the cell (dx, dy, dz) away from i's cell.
__device__ __forceinline__ uint32_t nbr_pack(int j, int dx, int dy, int dz) {
  return (uint32_t)j | (uint32_t)((dx + 1) | (dy + 1) << 2 | (dz + 1) << 4) << kNbrIdxBits;
}

// -(cell offset of entry e along axis a) * cs: the field holds d + 1 in
// {0, 1, 2}, so cs - (d + 1) cs is -d cs, exact (a bit-field extract, a
// conversion and one fused multiply-add).
template <typename T>
__device__ __forceinline__ T nbr_shift(uint32_t e, int a, T cs) {
  const uint32_t d1 = (e >> (kNbrIdxBits + 2 * a)) & 3u;
  return fma(-T(d1), cs, cs);
}

// The list entries a lane of a team takes: groups of V consecutive entries
// of one chunk, group g of lane l starting at entry L V g + V l.  V is the
// largest of 4, 2, 1 that divides the batch of U entries per lane and is at
// most C / L (one with C or more lanes: lane l takes l, l + L, ...), so that
// narrow teams read whole chunks with vector loads.
template <int DIM, int L, int U>
constexpr int list_vec() {
  constexpr int C = nbr_chunk<DIM>();
  constexpr int vmax = L >= C ? 1 : C / L;
  return (vmax >= 4 && U % 4 == 0) ? 4 : ((vmax >= 2 && U % 2 == 0) ? 2 : 1);
}

// Entry of element u of the batch that starts at group g0.
template <int DIM, int L, int U>
__device__ __forceinline__ int list_entry(int g0, int lane, int u) {
  constexpr int V = list_vec<DIM, L, U>();
  return L * V * (g0 + u / V) + V * lane + u % V;
}

// The U entries of lane `lane` in the batch that starts at group g0 (whose
// first entry is below cnt).  A group that starts at or past cnt re-reads
// the first one, so no load leaves the rows in use; elements past cnt are
// read but never used.
template <int DIM, int L, int U>
__device__ __forceinline__ void list_batch(const uint32_t* nbr, int64_t stride, int i, int lane,
                                           int g0, int cnt, uint32_t (&e)[U]) {
  constexpr int V = list_vec<DIM, L, U>();
  constexpr int NV = U / V;
  // every address first, then every load, so that the loads of a batch are
  // in flight together
  const uint32_t* p[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    int k = list_entry<DIM, L, U>(g0, lane, v * V);
    if (k >= cnt) k = list_entry<DIM, L, U>(g0, lane, 0);
    p[v] = nbr + nbr_index<DIM>(k, i, stride);
  }
  if constexpr (V == 4) {
    uint4 w[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) w[v] = *reinterpret_cast<const uint4*>(p[v]);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      e[4 * v] = w[v].x;
      e[4 * v + 1] = w[v].y;
      e[4 * v + 2] = w[v].z;
      e[4 * v + 3] = w[v].w;
    }
  } else if constexpr (V == 2) {
    uint2 w[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) w[v] = *reinterpret_cast<const uint2*>(p[v]);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      e[2 * v] = w[v].x;
      e[2 * v + 1] = w[v].y;
    }
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) e[v] = *p[v];
  }
}

// The particle gathered for element u of a batch: its entry while valid.
// Past the count, one-entry groups hold the batch's first entry (re-read by
// list_batch) and wider groups any value: both gather the first entry's j,
// which the lane loads anyway.
template <int DIM, int L, int U>
__device__ __forceinline__ int list_j(const uint32_t (&e)[U], int u, bool valid) {
  constexpr int V = list_vec<DIM, L, U>();
  return (int)(((V == 1 || valid) ? e[u] : e[0]) & kNbrIdxMask);
}

template <typename T, int DIM, int L, typename Fn>
__device__ __forceinline__ void for_neighbors(const PairCtx<T>& pc, int i, int lane,
                                              const T xi[3], Fn&& fn) {
  const int cnt = (pc.nbr && !(pc.stale && *pc.stale)) ? pc.ncnt[i] : kNbrNoList;
  if (cnt <= pc.nk) {   // a particle whose list overflowed scans the stencil
    constexpr int kG = kUnroll / list_vec<DIM, L, kUnroll>();   // groups per batch
    for (int g0 = 0; list_entry<DIM, L, kUnroll>(g0, lane, 0) < cnt; g0 += kG) {
      uint32_t e[kUnroll];
      list_batch<DIM, L, kUnroll>(pc.nbr, pc.nstride, i, lane, g0, cnt, e);
      T q0[kUnroll], q1[kUnroll], q2[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int j = list_j<DIM, L>(e, u, list_entry<DIM, L, kUnroll>(g0, lane, u) < cnt);
        q0[u] = pc.xr[0][j];
        q1[u] = pc.xr[1][j];
        q2[u] = DIM == 3 ? pc.xr[2][j] : T(0);
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        if (list_entry<DIM, L, kUnroll>(g0, lane, u) >= cnt) break;
        const int j = (int)(e[u] & kNbrIdxMask);
        T r[3];
        r[0] = (xi[0] - q0[u]) + nbr_shift<T>(e[u], 0, pc.csz);
        r[1] = (xi[1] - q1[u]) + nbr_shift<T>(e[u], 1, pc.csz);
        r[2] = DIM == 3 ? (xi[2] - q2[u]) + nbr_shift<T>(e[u], 2, pc.csz) : T(0);
        const T r2 = DIM == 3 ? (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]
                              : r[0] * r[0] + r[1] * r[1];
        if (r2 < pc.rc2) fn(j, r, r2);
      }
    }
    return;
  }
  const int c = pc.cell[i];
  const int cx = c % pc.nx;
  const int cyz = c / pc.nx;
  const int cy = cyz % pc.ny;
  const int cz = cyz / pc.ny;
  constexpr int zr = DIM == 3 ? 1 : 0;
#pragma unroll
  for (int dz = -zr; dz <= zr; ++dz) {
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const int base = ((cz + dz) * pc.ny + (cy + dy)) * pc.nx + cx;
      const int j0 = pc.cs[base - 1], j1 = pc.cs[base], j2 = pc.cs[base + 1],
                j3 = pc.cs[base + 2];
      const T oy = -T(dy) * pc.csz, oz = -T(dz) * pc.csz;
      for (int jb = j0 + lane; jb < j3; jb += kUnroll * L) {
        T q0[kUnroll], q1[kUnroll], q2[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int j = jb + u * L;
          const int js = j < j3 ? j : jb;
          q0[u] = pc.xr[0][js];
          q1[u] = pc.xr[1][js];
          q2[u] = DIM == 3 ? pc.xr[2][js] : T(0);
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int j = jb + u * L;
          if (j >= j3) break;
          const T ox = j < j1 ? pc.csz : (j < j2 ? T(0) : -pc.csz);
          T r[3];
          r[0] = (xi[0] - q0[u]) + ox;
          r[1] = (xi[1] - q1[u]) + oy;
          r[2] = DIM == 3 ? (xi[2] - q2[u]) + oz : T(0);
          const T r2 = DIM == 3 ? (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]
                                : r[0] * r[0] + r[1] * r[1];
          if (r2 < pc.rc2 && j != i) fn(j, r, r2);
        }
      }
    }
  }
}

// Record of particle j for the pressure pass: position, p, V (negative for
// a wall), correction matrix.  2D: {x0, x1, p, Vw} {Bxx, Bxy, Byy, 0};
// 3D: {x0, x1, x2, p} {Vw, Bxx, Bxy, Bxz} {Byy, Byz, Bzz, 0}.
template <typename T, int DIM>
__device__ __forceinline__ void write_prec(V4<T>* const* pr, int i, const T x[3], T p, T volw,
                                           const T B[6]) {
  if (DIM == 2) {
    pr[0][i] = V4<T>{x[0], x[1], p, volw};
    pr[1][i] = V4<T>{B[0], B[1], B[3], T(0)};
  } else {
    pr[0][i] = V4<T>{x[0], x[1], x[2], p};
    pr[1][i] = V4<T>{volw, B[0], B[1], B[2]};
    pr[2][i] = V4<T>{B[3], B[4], B[5], T(0)};
  }
}

// Record of particle j for the continuity pass: position, velocity, p, V
// (negative for a wall).  2D: {x0, x1, v0, v1} {p, Vw, p_lo, 0} where p_lo
// is what the FP64 pressure loses in its rounding to p (FP32 pairs: p + p_lo
// carries it to FP64 accuracy, so that a pressure difference of two
// neighbours keeps its digits; 0 in FP64);
// 3D: {x0, x1, x2, v0} {v1, v2, p, Vw}.
template <typename T, int DIM>
__device__ __forceinline__ void write_drec(V4<T>* const* dr, int i, const T x[3], const T v[3],
                                           T p, T volw, T plo = T(0)) {
  if (DIM == 2) {
    dr[0][i] = V4<T>{x[0], x[1], v[0], v[1]};
    dr[1][i] = V4<T>{p, volw, plo, T(0)};
  } else {
    dr[0][i] = V4<T>{x[0], x[1], x[2], v[0]};
    dr[1][i] = V4<T>{v[1], v[2], p, volw};
  }
}

#ifndef SPHX_PIN_RECORDS
#define SPHX_PIN_RECORDS 1
#endif
#ifndef SPHX_LAZY_MIN_NR
#define SPHX_LAZY_MIN_NR 2
#endif
#ifndef SPHX_LAZY_MIN_NR64
#define SPHX_LAZY_MIN_NR64 2
#endif
#ifndef SPHX_LAZY_MAX_NR
#define SPHX_LAZY_MAX_NR 1
#endif
#ifndef SPHX_LAZY_MAX_NR64
#define SPHX_LAZY_MAX_NR64 1
#endif
// Every vector of a batch's records is needed by then: left alone, the
// compiler sinks the parts a candidate's distance test does not read into
// the test's branch, where they cost a second memory round trip.  An empty
// asm statement that takes each register keeps all the loads in front of the
// tests (it emits no instruction).  Measured with FP32 records in 2D:
// pressure -4 to -6 % from 160k to 2.56M particles.  In 3D and with FP64
// records the registers it holds cost more than the round trip (3D
// continuity +24 % on the mixer, the FP64 U-channel step +4 %): left out.
#ifndef SPHX_PIN_3D
#define SPHX_PIN_3D 0
#endif
template <typename T, int DIM, int U, int NR>
__device__ __forceinline__ void pin_records(V4<T> (&q)[U][NR]) {
  if (!SPHX_PIN_RECORDS || (DIM == 3 && !SPHX_PIN_3D) || sizeof(T) != 4) return;
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int w = 0; w < NR; ++w)
      asm volatile("" : "+v"(q[u][w].a), "+v"(q[u][w].b), "+v"(q[u][w].c), "+v"(q[u][w].d));
}

// for_neighbors over j-side records: the NR record vectors of every
// candidate of a batch are loaded together (the first holds its position),
// then the candidates are tested; fn(j, r, r2, q) with q[0..NR-1] the
// records of j.  Same pairs in the same order as for_neighbors.
// The record passes carry less per candidate than the position-only loop:
// deeper batches pay off when few lanes share a particle (measured: 6 at one
// or two lanes); at four, with the next batch's entries loading under the
// current records, two candidates per lane and batch are best.  Two-lane
// teams over FP32 3D records take 8 (four chunks of the list per batch; the
// 3.75M-particle mixer: advection 1932 -> 1673 us, continuity 1853 -> 1541,
// pressure 2357 -> 2339), and 12 over two-vector records (continuity 1423
// -> 1342 us at three wavefronts per SIMD against four; 16: 1588 us at
// two); fewer candidates per batch for more resident wavefronts lost (6 / 4:
// pressure 2321 / 2386 against 2179 us).  With the relative-motion radius
// and whole records: pressure 8 (6: 1310, 10: 1383 against 1194 us), the
// two-vector records 10 (8: continuity 730, advection 905 us; 10: 708, 968;
// 12: 761, 1081).  FP64 3D ones keep 6 (pressure 3942 against 5374 us at
// 8).
#ifndef SPHX_REC_UNROLL_WIDE
#define SPHX_REC_UNROLL_WIDE 2
#endif
#ifndef SPHX_REC_UNROLL_NARROW
#define SPHX_REC_UNROLL_NARROW 6
#endif
#ifndef SPHX_REC_UNROLL_NARROW3
#define SPHX_REC_UNROLL_NARROW3 8
#endif
#ifndef SPHX_REC_UNROLL_NARROW3_NR2
#define SPHX_REC_UNROLL_NARROW3_NR2 10
#endif
#ifndef SPHX_REC_UNROLL_ONE
#define SPHX_REC_UNROLL_ONE 6
#endif
// Four-lane FP64 3D teams take deeper batches: 3 for the three-vector
// pressure records, 4 for two-vector ones (the FP64 mixer: pressure 2244 ->
// 2136 us at 3, 2489 at 4; continuity 1445 -> 1356 / 1331 us; advection with
// B 1667 -> 1618 / 1571 us; the 2D four-lane passes keep 2: the U-channel
// step 0.279 against 0.288 ms at 3).
#ifndef SPHX_REC_UNROLL_WIDE3_64
#define SPHX_REC_UNROLL_WIDE3_64 3
#endif
#ifndef SPHX_REC_UNROLL_WIDE3_64_NR2
#define SPHX_REC_UNROLL_WIDE3_64_NR2 4
#endif
template <typename T, int DIM, int L, int NR>
constexpr int rec_unroll() {
  if (L >= 4 && DIM == 3 && sizeof(T) == 8)
    return NR <= 2 ? SPHX_REC_UNROLL_WIDE3_64_NR2 : SPHX_REC_UNROLL_WIDE3_64;
  if (L >= 4) return SPHX_REC_UNROLL_WIDE;
  if (L == 1) return SPHX_REC_UNROLL_ONE;
  if (DIM == 3 && sizeof(T) == 4)
    return NR <= 2 ? SPHX_REC_UNROLL_NARROW3_NR2 : SPHX_REC_UNROLL_NARROW3;
  return SPHX_REC_UNROLL_NARROW;
}

// The start of a particle's walk of its list: the count, the stale word and
// the first batch of entries, loaded before the particle's tag is tested so
// that none of them waits for it.  Every one of the list's rows is
// allocated, so the first batch needs no count (entries past it are read
// and never used).
template <int U>
struct ListHead {
  int cnt;
  bool stale;
  uint32_t e[U];
};

// Teams of at least this many lanes load the head of the list with the tag;
// narrower ones load it in the walk.
#ifndef SPHX_HEAD_MIN_LANES
#define SPHX_HEAD_MIN_LANES 4
#endif
template <int L>
constexpr bool head_early() {
  return L >= SPHX_HEAD_MIN_LANES;
}

template <typename T, int DIM, int L, int NR>
__device__ __forceinline__ ListHead<rec_unroll<T, DIM, L, NR>()> list_head(const PairCtx<T>& pc,
                                                                           int i, int lane) {
  constexpr int U = rec_unroll<T, DIM, L, NR>();
  ListHead<U> h;
  h.cnt = 0;
  h.stale = true;
#pragma unroll
  for (int u = 0; u < U; ++u) h.e[u] = 0u;
  if (head_early<L>() && pc.nbr) {
    h.cnt = pc.ncnt[i];
    h.stale = pc.stale && *pc.stale;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = lane + u * L;
      h.e[u] = pc.nbr[nbr_index<DIM>(k < pc.nk ? k : pc.nk - 1, i, pc.nstride)];
    }
  }
  return h;
}

// Teams of at least SPHX_HOIST_MIN_LANES lanes issue the loads of the update
// after the sum before the walk.  Narrower teams walk more batches per lane,
// so the latency saved is smaller and the registers held through the walk
// cost occupancy (measured: 3D two-lane and 2D FP64 one-lane pressure passes
// fell below four and three wavefronts per SIMD).  Where the head of the list
// was loaded with the tag, SPHX_AHEAD_MIN_LANES bounds the teams that also
// load the next batch's entries under the current batch's records.
#ifndef SPHX_AHEAD_MIN_LANES
#define SPHX_AHEAD_MIN_LANES 1
#endif
// 3D teams of one or two lanes also load the next batch's list entries
// under the current batch's records (the 3.75M-particle mixer: FP32
// advection 1798 -> 1600 us, FP64 continuity 2826 -> 2700 us, the others
// level or 1-3 % faster).
#ifndef SPHX_AHEAD_NARROW3
#define SPHX_AHEAD_NARROW3 1
#endif
#ifndef SPHX_HOIST_MIN_LANES
#define SPHX_HOIST_MIN_LANES 4
#endif
template <int L>
constexpr bool hoist_epilogue() {
  return L >= SPHX_HOIST_MIN_LANES;
}

// The list walk proper.  Wide teams start from the head loaded with the tag
// and gather each batch's records while the next batch's entries load (a
// slot past the count gathers particle i's own records: in bounds, never
// used).  Narrow teams, whose lists span several batches per lane, load the
// count and each batch's entries in turn (measured: the early head made the
// 3D two-lane passes 11-18 % slower).
template <typename T, int DIM, int L, int NR, typename Fn>
__device__ __forceinline__ void for_neighbors_rec(const PairCtx<T>& pc, int i, int lane,
                                                  const T xi[3], const V4<T>* const* rec,
                                                  const ListHead<rec_unroll<T, DIM, L, NR>()>& h,
                                                  Fn&& fn) {
  constexpr int kUnroll = rec_unroll<T, DIM, L, NR>();
  constexpr bool kAhead = L >= SPHX_AHEAD_MIN_LANES;
  // the candidates of one batch: entries e, records q
  // 3D records span two or three vectors but about 40 % of the list's
  // candidates lie within 2h: a batch gathers the first vector (position) of
  // every candidate, tests them all, then gathers the rest of the accepted
  // candidates' records together and evaluates them.  The gathers, not the
  // arithmetic, bound the 3D passes.  Measured on the 3.75M-particle mixer:
  // FP32 pressure (three vectors) 2733 -> 2542 us, FP64 pressure 4942 ->
  // 4394 us, FP64 continuity 3118 -> 2706 us.  FP32 two-vector records
  // (continuity, laminar advection) lost with one-entry list rows and the
  // divided stencil code (continuity 1640 -> 1753 us) but gain with the
  // chunked list, its bit-field offsets and the batches of eight (advection
  // 1597 -> 1447 us, continuity 1551 -> 1419 us).  With the relative-
  // motion radius about 70 % of the ~100 entries lie within 2h, and the
  // records load whole again (each candidate's other vectors issued after
  // its own test): FP32 pressure 1382 -> 1195 us, FP64 mixer step 21.02 ->
  // 20.44 ms, and, once the advection pass also formed B, the FP32
  // two-vector passes in batches of 10 (continuity 761 -> 708 us, advection
  // 1081 -> 968 us).  The two rounds remain as an option (SPHX_LAZY_*).
  constexpr bool kLazy =
      DIM == 3 && NR >= (sizeof(T) == 8 ? SPHX_LAZY_MIN_NR64 : SPHX_LAZY_MIN_NR) &&
      NR <= (sizeof(T) == 8 ? SPHX_LAZY_MAX_NR64 : SPHX_LAZY_MAX_NR);
  auto load_batch = [&](V4<T> (&q)[kUnroll][NR], const int (&jv)[kUnroll]) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
#pragma unroll
      for (int w = 0; w < (kLazy ? 1 : NR); ++w) q[u][w] = rec[w][jv[u]];
  };
  auto test_lazy = [&](const bool (&valid)[kUnroll], const uint32_t (&e)[kUnroll],
                       V4<T> (&q)[kUnroll][NR]) {
    T rv[kUnroll][3], r2v[kUnroll];
    bool ok[kUnroll];
    int jv[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      jv[u] = (int)(e[u] & kNbrIdxMask);
      rv[u][0] = (xi[0] - q[u][0].a) + nbr_shift<T>(e[u], 0, pc.csz);
      rv[u][1] = (xi[1] - q[u][0].b) + nbr_shift<T>(e[u], 1, pc.csz);
      rv[u][2] = (xi[2] - q[u][0].c) + nbr_shift<T>(e[u], 2, pc.csz);
      r2v[u] = (rv[u][0] * rv[u][0] + rv[u][1] * rv[u][1]) + rv[u][2] * rv[u][2];
      ok[u] = valid[u] && r2v[u] < pc.rc2;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
      if (ok[u])
#pragma unroll
        for (int w = 1; w < NR; ++w) q[u][w] = rec[w][jv[u]];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
      if (ok[u]) fn(jv[u], rv[u], r2v[u], q[u]);
  };
  auto test = [&](const bool (&valid)[kUnroll], const uint32_t (&e)[kUnroll],
                  const V4<T> (&q)[kUnroll][NR]) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (!valid[u]) break;
      const int j = (int)(e[u] & kNbrIdxMask);
      T r[3];
      r[0] = (xi[0] - q[u][0].a) + nbr_shift<T>(e[u], 0, pc.csz);
      r[1] = (xi[1] - q[u][0].b) + nbr_shift<T>(e[u], 1, pc.csz);
      r[2] = DIM == 3 ? (xi[2] - q[u][0].c) + nbr_shift<T>(e[u], 2, pc.csz) : T(0);
      const T r2 = DIM == 3 ? (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]
                            : r[0] * r[0] + r[1] * r[1];
      if (r2 < pc.rc2) fn(j, r, r2, q[u]);
    }
  };
  if (!head_early<L>()) {
    // the count and each batch's entries after the tag test; a slot past
    // the count repeats the batch's first entry (an overflowed list: the
    // stencil below)
    const int cnt = (pc.nbr && !(pc.stale && *pc.stale)) ? pc.ncnt[i] : kNbrNoList;
    if (cnt <= pc.nk) {
      constexpr int kG = kUnroll / list_vec<DIM, L, kUnroll>();   // groups per batch
      constexpr bool kAheadN = SPHX_AHEAD_NARROW3 && DIM == 3;
      uint32_t e[kUnroll];
      if (kAheadN && cnt > 0 && list_entry<DIM, L, kUnroll>(0, lane, 0) < cnt)
        list_batch<DIM, L, kUnroll>(pc.nbr, pc.nstride, i, lane, 0, cnt, e);
      for (int g0 = 0; list_entry<DIM, L, kUnroll>(g0, lane, 0) < cnt; g0 += kG) {
        if (!kAheadN) list_batch<DIM, L, kUnroll>(pc.nbr, pc.nstride, i, lane, g0, cnt, e);
        V4<T> q[kUnroll][NR];
        int jv[kUnroll];
        bool valid[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          valid[u] = list_entry<DIM, L, kUnroll>(g0, lane, u) < cnt;
          jv[u] = list_j<DIM, L>(e, u, valid[u]);
        }
        load_batch(q, jv);
        // the next batch's entries load under this batch's records
        uint32_t en[kUnroll];
        if (kAheadN && list_entry<DIM, L, kUnroll>(g0 + kG, lane, 0) < cnt)
          list_batch<DIM, L, kUnroll>(pc.nbr, pc.nstride, i, lane, g0 + kG, cnt, en);
        if constexpr (kLazy) {
          test_lazy(valid, e, q);
        } else {
          pin_records<T, DIM, kUnroll, NR>(q);
          test(valid, e, q);
        }
        if (kAheadN) {
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) e[u] = en[u];
        }
      }
      return;
    }
  } else if (pc.nbr && !h.stale && h.cnt <= pc.nk) {
    const int cnt = h.cnt;
    uint32_t e[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) e[u] = h.e[u];
    for (int kb = lane; kb < cnt; kb += kUnroll * L) {
      if (!kAhead && kb != lane) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int k = kb + u * L;
          e[u] = k < cnt ? pc.nbr[nbr_index<DIM>(k, i, pc.nstride)] : 0u;
        }
      }
      V4<T> q[kUnroll][NR];
      int jv[kUnroll];
      bool valid[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        valid[u] = kb + u * L < cnt;
        jv[u] = valid[u] ? (int)(e[u] & kNbrIdxMask) : i;
      }
      load_batch(q, jv);
      uint32_t en[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int k = kb + (kUnroll + u) * L;
        en[u] = (kAhead && k < cnt) ? pc.nbr[nbr_index<DIM>(k, i, pc.nstride)] : 0u;
      }
      if constexpr (kLazy) {
        test_lazy(valid, e, q);
      } else {
        pin_records<T, DIM, kUnroll, NR>(q);
        test(valid, e, q);
      }
      if (kAhead) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) e[u] = en[u];
      }
    }
    return;
  }
  const int c = pc.cell[i];
  const int cx = c % pc.nx;
  const int cyz = c / pc.nx;
  const int cy = cyz % pc.ny;
  const int cz = cyz / pc.ny;
  constexpr int zr = DIM == 3 ? 1 : 0;
  for (int dz = -zr; dz <= zr; ++dz) {
    for (int dy = -1; dy <= 1; ++dy) {
      const int base = ((cz + dz) * pc.ny + (cy + dy)) * pc.nx + cx;
      const int j0 = pc.cs[base - 1], j1 = pc.cs[base], j2 = pc.cs[base + 1],
                j3 = pc.cs[base + 2];
      const T oy = -T(dy) * pc.csz, oz = -T(dz) * pc.csz;
      for (int jb = j0 + lane; jb < j3; jb += kUnroll * L) {
        V4<T> q[kUnroll][NR];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int j = jb + u * L;
          const int js = j < j3 ? j : jb;
#pragma unroll
          for (int w = 0; w < NR; ++w) q[u][w] = rec[w][js];
        }
        pin_records<T, DIM, kUnroll, NR>(q);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int j = jb + u * L;
          if (j >= j3) break;
          const T ox = j < j1 ? pc.csz : (j < j2 ? T(0) : -pc.csz);
          T r[3];
          r[0] = (xi[0] - q[u][0].a) + ox;
          r[1] = (xi[1] - q[u][0].b) + oy;
          r[2] = DIM == 3 ? (xi[2] - q[u][0].c) + oz : T(0);
          const T r2 = DIM == 3 ? (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]
                                : r[0] * r[0] + r[1] * r[1];
          if (r2 < pc.rc2 && j != i) fn(j, r, r2, q[u]);
        }
      }
    }
  }
}

// Output of a neighbour-list build.
template <typename T>
struct NbrOut {
  uint32_t* nbr;
  int32_t* ncnt;
  int64_t stride;
  int K;
  T* xb[3];
  uint32_t* flags;
  uint32_t* stale;
  T rl2;
  uint32_t* stage;   // LDS rows of this particle's first kstage entries (NULL: none)
  int kstage;
  V4<T>* queue;      // LDS pair queue of this wavefront (pair_queue entries per lane)
  // relative-motion radius (tight, with lrad[0] = the step's Δt_ad > 0): j is
  // listed when |r_ij| < 2h + s_i + s_j + |u_c(i) - u_c(j)| Δt_ad (a wall's
  // s_j = |u_c(j)| Δt_ad), at most the cell size rl; otherwise when |r_ij| < rl
  int tight;
  double* lrad;
  const float* lskin;
  const T* cell_u[3];
  // FP32 copies of the cell-relative positions (FP64 contexts; else NULL)
  const float* xs[3];
  T two_h, rl;
  // starts of the x quarters 1-3 of every cell (NULL: whole rows), q_rl a
  // little above rl, q_w = 4 / cell size
  const int32_t* cell_q;
  T q_rl, q_w;
};

// Pairs within 2h found by the 3D FP32 list build wait in a per-lane queue
// in LDS ({r, V_j}, 16 bytes) and their terms are evaluated when some lane's
// queue is full, all queued pairs of the wavefront together.  Evaluated in
// the scan itself, the terms ran for nearly every candidate batch (one lane
// or another of the wavefront always had a pair within 2h, about 7 % of the
// ~1000 candidates), at about a third of the scan's instructions.  Each lane
// still takes its pairs in the order it found them.  Q entries per lane take
// Q KB of LDS per wavefront: up to 7 keep five 256-lane workgroups per CU.
// The 3.75M-particle mixer: 5106 us without the queue, 5102 / 5079 / 5017 us
// with 4 / 6 / 7 entries (6 % fewer VALU instructions; a queue fills about
// every 35 candidates somewhere in the wavefront).
#ifndef SPHX_PAIR_QUEUE
#define SPHX_PAIR_QUEUE 7
#endif
template <typename T, int DIM>
constexpr int pair_queue() {
  return (DIM == 3 && sizeof(T) == 4) ? SPHX_PAIR_QUEUE : 0;
}

// |r|^2 as every pass forms it
template <typename T, int DIM>
__device__ __forceinline__ T dist2(const T r[3]) {
  return DIM == 3 ? (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2] : r[0] * r[0] + r[1] * r[1];
}

#ifndef SPHX_LIST_STAGE
#define SPHX_LIST_STAGE 1
#endif
// The 2D list's one-entry rows make a wavefront's reads of entry k one
// line, but its appends scattered: each particle of a wavefront appends at
// its own count, a different row.  With four or more lanes per particle
// (2D, up to 260k particles) the entries are collected in LDS (16 KB or less
// per workgroup) and written out row by row at the end of the scan: the
// correction took 27.3 against 28.5 us at 57.6k particles and 57.3 against
// 58.6 us at 160k.  With fewer lanes the 32-48 KB of LDS cost more
// residency than the scattered stores (178 against 161 us at 640k).  3D
// appends go straight to the list, whose four-entry chunks keep a particle's
// appends within a few lines.
template <int DIM, int L>
constexpr int list_stage() {
  return (SPHX_LIST_STAGE && DIM == 2 && L >= 4) ? kNbrMax2 : 0;
}

// Candidates per lane and batch of the stencil scan: the position-only
// loop's, or SPHX_SCAN_UNROLL3 for the 3D scan that writes the list alone
// (the mixer: 3 and 4 level with 2).
#ifndef SPHX_SCAN_UNROLL3
#define SPHX_SCAN_UNROLL3 2
#endif
template <int DIM, int QD>
constexpr int scan_unroll() {
  return (DIM == 3 && QD == 0) ? SPHX_SCAN_UNROLL3 : kUnroll;
}

// Cell-stencil scan of particle i that also writes its neighbour list: every
// j != i with |r_ij|^2 < rl2 (rl = cell size, a little above to cover
// rounding), in stencil order.  A team of L lanes scans a row together (lane
// l takes every L-th candidate, in the order of for_neighbors) and appends
// the accepted candidates in candidate order with a wavefront ballot, so the
// list order does not depend on L.  fn(j, r, r2, V_j) is called for the
// pairs within 2h, in for_neighbors' order.
template <typename T, int DIM, int L, int QD = pair_queue<T, DIM>(), bool LO = false,
          typename Fn>
__device__ __forceinline__ void scan_build(const PairCtx<T>& pc, int i, int lane, const T xi[3],
                                           const NbrOut<T>& o, Fn&& fn) {
  // The FP64 scan that writes the list alone (LO) tests in FP32, on the
  // cell build's FP32 copies of the cell-relative positions: the list needs
  // every pair within its radius, and the radius's margin (2e-5 relative,
  // 2e-6 at the cell-size cap) is far above FP32's rounding of r.  Only the
  // passes' own FP64 test decides a pair.
  constexpr bool kS32 = LO && sizeof(T) == 8;
  using S = typename std::conditional<kS32, float, T>::type;
  const S* px[3];
  S xs[3];
  if constexpr (kS32) {
#pragma unroll
    for (int k = 0; k < 3; ++k) px[k] = o.xs[k];
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) px[k] = pc.xr[k];
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) xs[k] = (kS32 && k < DIM) ? px[k][i] : (S)xi[k];
  const S csz = (S)pc.csz, rl = (S)o.rl, rl2 = (S)o.rl2;
  const int wl = (int)(threadIdx.x & (kWave - 1));
  const int team0 = wl - lane;   // first lane of the team in the wavefront
  const uint64_t tmask = (L >= kWave ? ~0ull : ((1ull << L) - 1ull)) << team0;
  const int c = pc.cell[i];
  const int cx = c % pc.nx;
  const int cyz = c / pc.nx;
  const int cy = cyz % pc.ny;
  const int cz = cyz / pc.ny;
  constexpr int zr = DIM == 3 ? 1 : 0;
  // relative-motion radius (NbrOut): i's part of the bound
  const bool tight = o.tight && o.lrad[0] > 0.0;
  S rad_i = rl, uc_i[3] = {S(0), S(0), S(0)}, dt_l = S(0);
  if (tight) {
    dt_l = (S)o.lrad[0];
    rad_i = (S)o.two_h + (S)o.lskin[i];
#pragma unroll
    for (int k = 0; k < DIM; ++k) uc_i[k] = (S)o.cell_u[k][c];
  }
  // The cell build orders every cell by quarter along x: the members of the
  // row's cell at +1 in quarters k_hi and above, and of the cell at -1 in
  // quarters below k_lo, lie farther than q_rl along x (quarter k of the
  // cell at +1 starts cs / 2 + k cs / 4 above i's cell centre), so each row
  // is one shorter contiguous range: 2.25 cells instead of 3
  int k_lo = 0, k_hi = 4;
  if (o.cell_q) {
    const S a_hi = ((S)o.q_rl + xs[0] - S(0.5) * csz) * (S)o.q_w;
    const S a_lo = (xs[0] + S(1.5) * csz - (S)o.q_rl) * (S)o.q_w;
    k_hi = (int)ceil(a_hi);
    k_lo = (int)floor(a_lo);
    k_hi = k_hi < 0 ? 0 : (k_hi > 4 ? 4 : k_hi);
    k_lo = k_lo < 0 ? 0 : (k_lo > 4 ? 4 : k_lo);
  }
  const int ql_k = k_lo > 0 ? k_lo - 1 : 0, qh_k = k_hi > 0 ? k_hi - 1 : 0;
  constexpr int Q = QD;
  constexpr int SU = scan_unroll<DIM, QD>();
  int qn = 0;   // this lane's queued pairs
  // the queued pairs' terms, in the order the lane found them (wavefront-
  // uniform call: every lane with a queued pair takes part)
  auto flush = [&]() {
#pragma unroll
    for (int k = 0; k < (Q > 0 ? Q : 1); ++k) {
      if (k < qn) {
        const V4<T> e = o.queue[k * kWave + wl];
        const T r[3] = {e.a, e.b, e.c};
        fn(0, r, dist2<T, DIM>(r), e.d);
      }
    }
    qn = 0;
  };
  int cnt = 0;
  for (int dz = -zr; dz <= zr; ++dz) {
    // the cell ranges of the plane's three rows, loaded together (the list
    // stores of a row would otherwise keep the next row's loads behind it)
    int rows[3][4], rq[3][2];
#pragma unroll
    for (int r3 = 0; r3 < 3; ++r3) {
      const int base = ((cz + dz) * pc.ny + (cy + r3 - 1)) * pc.nx + cx;
#pragma unroll
      for (int k = 0; k < 4; ++k) rows[r3][k] = pc.cs[base - 1 + k];
      rq[r3][0] = rq[r3][1] = 0;
      if (o.cell_q) {
        rq[r3][0] = o.cell_q[4 * (int64_t)(base - 1) + ql_k];
        rq[r3][1] = o.cell_q[4 * (int64_t)(base + 1) + qh_k];
      }
    }
#pragma unroll
    for (int r3 = 0; r3 < 3; ++r3) {
      const int dy = r3 - 1;
      const int j0 = rows[r3][0], j1 = rows[r3][1], j2 = rows[r3][2], j3 = rows[r3][3];
      // the row's range within reach (an empty cell's quarter starts are not
      // written: clamped to the cell)
      int lo = j0, hi = j3;
      if (o.cell_q) {
        const int ql = rq[r3][0] < j0 ? j0 : (rq[r3][0] > j1 ? j1 : rq[r3][0]);
        const int qh = rq[r3][1] < j2 ? j2 : (rq[r3][1] > j3 ? j3 : rq[r3][1]);
        lo = k_lo == 0 ? j0 : ql;
        hi = k_hi == 0 ? j2 : qh;
      }
      const S oy = -S(dy) * csz, oz = -S(dz) * csz;
      // |u_c(i) - u_c| Δt_ad for the row's three cells
      S du[3] = {S(0), S(0), S(0)};
      if (tight) {
        const int cb = ((cz + dz) * pc.ny + (cy + dy)) * pc.nx + cx - 1;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          S d[3] = {S(0), S(0), S(0)};
#pragma unroll
          for (int k = 0; k < DIM; ++k) d[k] = uc_i[k] - (S)o.cell_u[k][cb + q];
          du[q] = pair_dist(DIM == 3 ? (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
                                     : d[0] * d[0] + d[1] * d[1]) * dt_l;
        }
      }
      // the same trip count for every lane of the team
      for (int jb = lo; jb < hi; jb += SU * L) {
        S q0[SU], q1[SU], q2[SU], qs[SU];
        T qv[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u) {
          const int j = jb + u * L + lane;
          // (an index below 2^26: 32-bit offsets from the arrays' bases)
          const uint32_t js = (uint32_t)(j < hi ? j : jb) & kNbrIdxMask;
          q0[u] = px[0][js];
          q1[u] = px[1][js];
          q2[u] = DIM == 3 ? px[2][js] : S(0);
          // with the positions: one round trip per batch
          qv[u] = LO ? T(0) : pc.vol[js];
          qs[u] = tight ? (S)o.lskin[js] : S(0);
        }
#pragma unroll
        for (int u = 0; u < SU; ++u) {
          const int j = jb + u * L + lane;
          const int dx = j < j1 ? -1 : (j < j2 ? 0 : 1);
          const S ox = j < j1 ? csz : (j < j2 ? S(0) : -csz);
          S r[3];
          r[0] = (xs[0] - q0[u]) + ox;
          r[1] = (xs[1] - q1[u]) + oy;
          r[2] = DIM == 3 ? (xs[2] - q2[u]) + oz : S(0);
          const S r2 = dist2<S, DIM>(r);
          const bool in = j < hi && j != i;
          S rad2 = rl2;
          if (tight) {
            // a little above for rounding, at most the cell size
            const S dux = dx < 0 ? du[0] : (dx == 0 ? du[1] : du[2]);
            const S rc = fmin((rad_i + qs[u] + dux) * S(1.00002), rl);
            rad2 = rc * rc;
          }
          const bool acc = in && r2 < rad2;
          int off = 0, tot = acc ? 1 : 0;
          if (L > 1) {
            // accepted lanes of the team; off = those below this lane
            const uint64_t tm = (uint64_t)__ballot(acc) & tmask;
            off = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(tm >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)tm, 0u));
            tot = __popcll(tm);
          }
          if (acc && cnt + off < o.K) {
            const uint32_t ent = nbr_pack(j, dx, dy, dz);
            if (list_stage<DIM, L>() > 0 && cnt + off < o.kstage) o.stage[cnt + off] = ent;
            else o.nbr[nbr_index<DIM>(cnt + off, i, o.stride)] = ent;
          }
          cnt += tot;
          if constexpr (LO) {
            // the list alone
          } else if constexpr (Q > 0) {
            if (in && r2 < pc.rc2) {
              o.queue[qn * kWave + wl] = V4<T>{r[0], r[1], r[2], qv[u]};
              ++qn;
            }
            if (__ballot(qn == Q)) flush();
          } else {
            if (in && r2 < pc.rc2) fn(j, r, r2, qv[u]);
          }
        }
      }
    }
  }
  if constexpr (Q > 0 && !LO) flush();
  // more candidates than the list holds (a particle in a cluster denser
  // than the lattice): the passes scan the stencil for this particle
  if (lane == 0) o.ncnt[i] = cnt <= o.K ? cnt : kNbrNoList;
  if (o.kstage > 0) {
    // the team's lanes wrote the staged entries; LDS operations of one
    // wavefront complete in order, the barrier keeps the compiler's order
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int m = cnt < o.kstage ? cnt : o.kstage;
    for (int k = lane; k < m; k += L) o.nbr[nbr_index<DIM>(k, i, o.stride)] = o.stage[k];
  }
}

// Start of a list build for particle i: its reference position and, for
// particles that are not real, an empty list.  Returns false for those.
template <typename T, int DIM>
__device__ __forceinline__ bool build_begin(const PairCtx<T>& pc, int i, int lane,
                                            const NbrOut<T>& o) {
  if (lane == 0) {
    o.xb[0][i] = pc.xr[0][i];
    o.xb[1][i] = pc.xr[1][i];
    if (DIM == 3) o.xb[2][i] = pc.xr[2][i];
  }
  if (!is_real(pc.tag[i])) {
    if (lane == 0) o.ncnt[i] = 0;
    return false;
  }
  return true;
}

// B (symmetric, packed xx xy xz yy yz zz) times a vector.
template <typename T, int DIM>
__device__ __forceinline__ void symv(const T B[6], const T a[3], T o[3]) {
  if (DIM == 2) {
    o[0] = B[0] * a[0] + B[1] * a[1];
    o[1] = B[1] * a[0] + B[3] * a[1];
    o[2] = T(0);
  } else {
    o[0] = B[0] * a[0] + B[1] * a[1] + B[2] * a[2];
    o[1] = B[1] * a[0] + B[3] * a[1] + B[4] * a[2];
    o[2] = B[2] * a[0] + B[4] * a[1] + B[5] * a[2];
  }
}

template <typename T, int DIM>
__device__ __forceinline__ void load_B(const T* const* Bp, int i, T B[6]) {
  B[0] = Bp[0][i];
  B[1] = Bp[1][i];
  B[3] = Bp[3][i];
  if (DIM == 3) {
    B[2] = Bp[2][i];
    B[4] = Bp[4][i];
    B[5] = Bp[5][i];
  } else {
    B[2] = B[4] = B[5] = T(0);
  }
}

// The 2D pressure pass in FP32 evaluates the kernel function in FP64: its
// sum cancels to a small fraction of its terms, and the FP32 kernel
// polynomial's rounding is the largest part of its error against FP64 (the
// pass has idle VALU cycles in 2D).
template <typename T, int DIM>
constexpr bool f64_kernel() {
  return DIM == 2 && sizeof(T) == 4;
}

// (dW/dr)/r and r of a pair in FP64 from its offset components in T:
// r^2 from exact FP64 squares, 1/r from the FP32 reciprocal square root
// refined by one Newton step in FP64 (relative error ~1e-14).
template <typename T>
__device__ __forceinline__ double dw_over_r_d(const T r[3], double inv_h, double kf,
                                              double* rr) {
  const double r0 = (double)r[0], r1 = (double)r[1];
  const double r2 = r0 * r0 + r1 * r1;
  double q = 0.0;
  if (r2 > 0.0) {
    const double y0 = (double)rsqrtf((float)r2);
    const double y = y0 * (1.5 - 0.5 * r2 * y0 * y0);
    q = r2 * y;
  }
  *rr = q;
  const double t = 1.0 - 0.5 * q * inv_h;
  return kf * t * t * t;
}

__device__ __forceinline__ double eos(double rho, double k, double rho0, double c0, int turb) {
  double p = rho0 * c0 * c0 * (rho / rho0 - 1.0);
  if (turb) p += (2.0 / 3.0) * rho * k;
  return p;
}

// B = A^-1 for a well-conditioned moment; with d = det A / (tr A / dim)^dim
// below 0.25 the inverse is blended towards the identity with weight
// (d / 0.25)^2, and B = I when tr A <= 0 or d <= 0.
template <int DIM>
__device__ __forceinline__ void invert_sym(const double A[6], double B[6]) {
  constexpr double theta = 0.25;
  // every branch leaves its values in registers and B is written once (an
  // early return with its own stores made the compiler keep B in scratch)
  double inv[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double det, tr, d;
  if (DIM == 2) {
    tr = A[0] + A[3];
    det = A[0] * A[3] - A[1] * A[1];
    d = tr > 0.0 ? det / ((0.5 * tr) * (0.5 * tr)) : 0.0;
    inv[0] = A[3] / det; inv[1] = -A[1] / det; inv[3] = A[0] / det;
  } else {
    const double c00 = A[3] * A[5] - A[4] * A[4];
    const double c01 = A[4] * A[2] - A[1] * A[5];
    const double c02 = A[1] * A[4] - A[3] * A[2];
    det = A[0] * c00 + A[1] * c01 + A[2] * c02;
    tr = A[0] + A[3] + A[5];
    const double t3 = tr / 3.0;
    d = tr > 0.0 ? det / (t3 * t3 * t3) : 0.0;
    inv[0] = c00 / det;
    inv[1] = c01 / det;
    inv[2] = c02 / det;
    inv[3] = (A[0] * A[5] - A[2] * A[2]) / det;
    inv[4] = (A[2] * A[1] - A[0] * A[4]) / det;
    inv[5] = (A[0] * A[3] - A[1] * A[1]) / det;
  }
  // guard: no positive trace or determinant -> B = I
  const bool ok = tr > 0.0 && d > 0.0;
  const double w = d >= theta ? 1.0 : (d / theta) * (d / theta);
  const double id[6] = {1.0, 0.0, 0.0, 1.0, 0.0, DIM == 3 ? 1.0 : 0.0};
#pragma unroll
  for (int k = 0; k < 6; ++k) B[k] = ok ? w * inv[k] + (1.0 - w) * id[k] : id[k];
}


template <typename T>
inline Consts<T> make_consts(const sph_ctx* c) {
  Consts<T> C;
  const sph_params& P = c->P;
  C.dim = P.dim;
  C.turbulence = P.turbulence;
  C.obc_mode = P.obc_mode;
  C.nbuf = c->nbuf;
  C.grid = c->grid;
  C.h = P.h;
  const double rc = 2.0 * P.h;
  C.rc2 = rc * rc;
  C.dp = P.dp;
  C.Vw = P.dim == 2 ? P.dp * P.dp : P.dp * P.dp * P.dp;
  C.mass = P.rho0 * C.Vw;
  C.rho0 = P.rho0;
  C.c0 = P.c0;
  C.nu_l = P.nu_l;
  C.eta = P.eta;
  for (int k = 0; k < 3; ++k) C.g[k] = P.g[k];
  C.C1 = P.C1;
  C.C2 = P.C2;
  C.Cmu = P.Cmu;
  C.sigma_k = P.sigma_k;
  C.sigma_eps = P.sigma_eps;
  C.k_floor = P.k_floor;
  C.eps_floor = P.eps_floor;
  C.skin = 0.5 * (P.cell_size - 2.0 * P.h);
  C.seed = P.seed;
  const double alpha = P.dim == 2 ? 7.0 / (4.0 * M_PI * P.h * P.h)
                                  : 21.0 / (16.0 * M_PI * P.h * P.h * P.h);
  C.h_t = (T)P.h;
  C.rc2_t = (T)C.rc2;
  C.cs_t = (T)P.cell_size;
  C.inv_h_t = (T)(1.0 / P.h);
  C.kf_t = (T)(-5.0 * alpha / (P.h * P.h));
  C.inv_h_d = 1.0 / P.h;
  C.kf_d = -5.0 * alpha / (P.h * P.h);
  C.rho0_t = (T)P.rho0;
  C.c0_t = (T)P.c0;
  C.eta_t = (T)P.eta;
  C.inv_2rc0_t = (T)(1.0 / (2.0 * P.rho0 * P.c0));
  C.mu_R_t = (T)(0.5 * P.rho0 * P.h);
  return C;
}

template <typename T>
inline PairCtx<T> make_pc(const sph_ctx* c, const sphx::Slot2<void>* xr, int xslot) {
  PairCtx<T> pc;
  for (int k = 0; k < 3; ++k) pc.xr[k] = tp<T>(xr[k].a[xslot]);
  pc.vol = tp<T>(c->F.vol.live());
  pc.tag = c->F.tag.live();
  pc.cell = c->F.cell;
  pc.cs = c->S.cell_start;
  pc.nx = c->grid.n[0];
  pc.ny = c->grid.n[1];
  pc.csz = (T)c->P.cell_size;
  const double rc = 2.0 * c->P.h;
  pc.rc2 = (T)(rc * rc);
  pc.inv_h = (T)(1.0 / c->P.h);
  pc.kf = T(0);
  pc.pairs = c->S.pairs;
  const bool list = c->use_nbr && c->nbr_valid;
  pc.nbr = list ? c->F.nbr : nullptr;
  pc.ncnt = list ? c->F.ncnt : nullptr;
  pc.nstride = c->cap;
  pc.nk = c->F.nbr_k;
  pc.stale = nullptr;
  return pc;
}

}  // namespace sphx
