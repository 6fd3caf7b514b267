// Device-side building blocks of the free-surface LBM step for gfx950:
// lattice tables, cell flags, population storage codecs, neighbour resolution,
// collision. Everything here is header-only and templated on the lattice (Q),
// the storage format (S) and the collision operator (TRT) so that the direction
// loops unroll into immediate offsets.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fslbm {

// ---------------------------------------------------------------------------
// Velocity sets (Sec. 2.1). Direction k: rest; +-x, +-y, +-z; the twelve edge
// directions; the eight corners. D3Q19 uses k < 19, D3Q27 all 27. Opposite
// pairs are (1,2), (3,4), ..., (25,26). The order is part of the exported
// population layout.
// ---------------------------------------------------------------------------
constexpr int kCX[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0,
                         1, -1, 1, -1, 1, -1, -1, 1};
constexpr int kCY[27] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1,
                         1, -1, 1, -1, -1, 1, 1, -1};
constexpr int kCZ[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1,
                         1, -1, -1, 1, 1, -1, 1, -1};

// Components of direction k (k may be a run-time value).
__host__ __device__ constexpr int cxd(int k) { return kCX[k]; }
__host__ __device__ constexpr int cyd(int k) { return kCY[k]; }
__host__ __device__ constexpr int czd(int k) { return kCZ[k]; }

__host__ __device__ constexpr int opp(int k) { return k == 0 ? 0 : ((k & 1) ? k + 1 : k - 1); }

template <int Q>
__host__ __device__ constexpr double weight(int k) {
  return Q == 19
             ? (k == 0 ? 1.0 / 3.0 : (k < 7 ? 1.0 / 18.0 : 1.0 / 36.0))
             : (k == 0 ? 8.0 / 27.0 : (k < 7 ? 2.0 / 27.0 : (k < 19 ? 1.0 / 54.0 : 1.0 / 216.0)));
}

// ---------------------------------------------------------------------------
// Cell flags: one byte per cell.
//   bits 0-2 type: gas, interface, liquid, no-slip obstacle, free-slip obstacle
//   bit 3 BORDER   (static) the 3x3x3 neighbourhood leaves the domain or holds
//                  an obstacle: neighbour lookups need wrap/wall handling
//   bit 4 NEW_GAS  became interface from gas in the last conversion
//   bit 5 NEW_LIQ  became interface from liquid in the last conversion
//   bit 6 CONV     interface cell converted to liquid or gas in the last conversion
//   bit 7 COMPLEX  (static) the 3x3x3 neighbourhood wraps through a periodic
//                  face, crosses a free-slip face or holds an obstacle cell; a
//                  BORDER cell without it only meets no-slip domain faces
// ---------------------------------------------------------------------------
enum : uint8_t { T_GAS = 0, T_IF = 1, T_LIQ = 2, T_NOSLIP = 3, T_FREESLIP = 4 };
constexpr uint8_t T_MASK = 7;
constexpr uint8_t F_BORDER = 8;
constexpr uint8_t F_NEW_GAS = 16;
constexpr uint8_t F_NEW_LIQ = 32;
constexpr uint8_t F_CONV = 64;
constexpr uint8_t F_COMPLEX = 128;
constexpr uint8_t F_TRANSIENT = F_NEW_GAS | F_NEW_LIQ | F_CONV;
constexpr uint8_t F_STATIC = F_BORDER | F_COMPLEX;

__host__ __device__ inline bool is_obst(int t) { return t == T_NOSLIP || t == T_FREESLIP; }
__host__ __device__ inline bool is_fluid(int t) { return t == T_IF || t == T_LIQ; }

enum : uint8_t { MK_NONE = 0, MK_L = 1, MK_G = 2 };
enum : uint8_t { CLS_STD = 0, CLS_NOLIQ = 1, CLS_NOGAS = 2 };
enum { BND_PERIODIC = 0, BND_NOSLIP = 1, BND_FREESLIP = 2 };

// Counter slots in device memory.
enum {
  CNT_IF = 0,      // interface cells in the list
  CNT_CONV = 1,    // converted cells in the list
  CNT_MARK0 = 2,   // marked cells, slot (step & 1)
  CNT_TICKET = 4,  // block tickets of the compaction scan
  CNT_ERR = 5,     // error bits (see ERR_*)
  CNT_EPOCH = 6,   // epoch of the compaction scan (advanced before every compaction)
  CNT_CHUNKS = 7,  // 64-cell chunks holding at least one liquid cell
  CNT_GEN = 8,     // liquid cells next to the domain boundary or an obstacle
  CNT_NG = 9,      // new interface cells from gas in this step
  CNT_HALT0 = 10,  // halt words, slot (step & 1): the run stopped after an instability
  CNT_NL = 12,     // new interface cells from liquid in this step
  CNT_SBASE = 13,  // in place: interface cells of this step (stash entries written by the step)
  CNT_SNEW = 14,   // in place: stash entries taken by this step's new interface cells
  CNT_SMOOTH = 15, // surface tension: smoothing-tile tag of this step, minus one
  CNT_N = 16
};
// ERR_STASH: in-place layout, more interface cells than a stash buffer holds;
// ERR_SLOTS: in-place layout, two (cell, direction) pairs stream through one slot
enum { ERR_UNSTABLE = 1, ERR_LAYER = 2, ERR_SCAN = 4, ERR_TYPE = 8, ERR_BUBBLE = 16, ERR_STASH = 32,
       ERR_SLOTS = 64 };

// ---------------------------------------------------------------------------
// Order-free sums (tracked-bubble totals). A value x is kept as hi = floor(x)
// (int64) and lo = (x - hi) 2^64 (uint64, rounded toward zero); the parts of
// many values are added as integers, exactly (lo modulo 2^64, its carries
// into hi), so a total built from atomic adds does not depend on their order.
// It is read back as hi + lo 2^-64 (two roundings, the same on host and
// device). Totals must stay below 2^63 in magnitude.
// ---------------------------------------------------------------------------
__host__ __device__ inline double fix_value(int64_t hi, uint64_t lo) {
  return (double)hi + (double)lo * 0x1p-64;
}

// ---------------------------------------------------------------------------
// Population storage. R is the arithmetic type; kShift tells whether the
// values handled by the kernels are f_k or h_k = f_k - w_k.
// ---------------------------------------------------------------------------
enum { ST_F64 = 0, ST_F32 = 1, ST_F16S = 2 };

template <int S, int Q>
struct Store;

// F64 keeps f itself (binary64 arithmetic, the reference path). The FP32
// formats keep the shifted population h_k = f_k - w_k: near rest f_k is close to
// its weight, so h_k carries the significant digits, and mass sums 1 + sum h
// do not pick up the rounding of the weights. F32 stores h in binary32, F16S in
// binary16 (round to nearest even); arithmetic is binary32 in both.
// ld/st address element o of a grid; bld/bst go through a raw buffer
// resource with a per-lane byte offset and a uniform (scalar) byte offset, so
// a cell's q loads share one address register.
template <int Q>
struct Store<ST_F64, Q> {
  using T = double;
  using R = double;
  static constexpr bool kShift = false;
  static __device__ __forceinline__ R ld(const T* p, int64_t o, int) { return p[o]; }
  static __device__ __forceinline__ void st(T* p, int64_t o, int, R v) { p[o] = v; }
  static __device__ __forceinline__ R bld(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, v, s, 0));
  }
  static __device__ __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s, R x) {
    using u2 = unsigned int __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, x), r, v, s, 0);
  }
};

template <int Q>
struct Store<ST_F32, Q> {
  using T = float;
  using R = float;
  static constexpr bool kShift = true;
  static __device__ __forceinline__ R ld(const T* p, int64_t o, int) { return p[o]; }
  static __device__ __forceinline__ void st(T* p, int64_t o, int, R v) { p[o] = v; }
  static __device__ __forceinline__ R bld(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0));
  }
  static __device__ __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s, R x) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, x), r, v, s, 0);
  }
};

template <int Q>
struct Store<ST_F16S, Q> {
  using T = _Float16;
  using R = float;
  static constexpr bool kShift = true;
  static __device__ __forceinline__ R ld(const T* p, int64_t o, int) {
    return static_cast<float>(p[o]);
  }
  static __device__ __forceinline__ void st(T* p, int64_t o, int, R v) {
    p[o] = static_cast<_Float16>(v);
  }
  static __device__ __forceinline__ R bld(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s) {
    return static_cast<float>(
        __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, v, s, 0)));
  }
  static __device__ __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s, R x) {
    __builtin_amdgcn_raw_buffer_store_b16(
        __builtin_bit_cast(unsigned short, static_cast<_Float16>(x)), r, v, s, 0);
  }
};

// Raw buffer resource over `bytes` bytes at p (range-checked: loads beyond
// return 0, stores beyond are dropped). Third dword as for the gfx9 family.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

// ---------------------------------------------------------------------------
// Geometry and neighbour lookup.
// ---------------------------------------------------------------------------
struct Geom {
  int nx, ny, nz;
  int bnd[6];
  uint32_t bnd_bits;  // bnd[f] in bits 2f, 2f+1
  int64_t N;       // nx*ny*nz
  int64_t stride;  // distance between population planes (>= N)
};

// Boundary kind of a face with a run-time face index, from the packed copy
// (an indexed load from bnd[] would make the whole kernel-argument block a
// private array).
__device__ __forceinline__ int face_kind(const Geom& g, int face) {
  return (int)((g.bnd_bits >> (2 * face)) & 3u);
}

// Cell coordinates; domains hold fewer than 2^30 cells, so 32-bit unsigned
// arithmetic suffices.
__device__ __forceinline__ void coords(const Geom& g, int64_t c, int& x, int& y, int& z) {
  const uint32_t cc = (uint32_t)c, nx = (uint32_t)g.nx, nxy = nx * (uint32_t)g.ny;
  const uint32_t zz = cc / nxy;
  const uint32_t r = cc - zz * nxy;
  const uint32_t yy = r / nx;
  z = (int)zz;
  y = (int)yy;
  x = (int)(r - yy * nx);
}

// Index of (x,y,z)+(dx,dy,dz) after periodic wrap, or -1 beyond a wall face;
// *wall receives the ghost's obstacle type (no-slip wins where faces meet).
// (x,y,z) is a cell of the domain and the offsets are -1, 0 or 1, so a
// periodic wrap is one period, and with compile-time offsets (directions of
// an unrolled loop) only the faces the offset can cross are tested; this
// keeps the function small, which matters where it is unrolled over q
// directions.
__device__ __forceinline__ int64_t nb_index(const Geom& g, int x, int y, int z, int dx, int dy,
                                            int dz, int* wall) {
  __builtin_assume(x >= 0 && x < g.nx);
  __builtin_assume(y >= 0 && y < g.ny);
  __builtin_assume(z >= 0 && z < g.nz);
  __builtin_assume(dx >= -1 && dx <= 1);
  __builtin_assume(dy >= -1 && dy <= 1);
  __builtin_assume(dz >= -1 && dz <= 1);
  int c[3] = {x + dx, y + dy, z + dz};
  const int n[3] = {g.nx, g.ny, g.nz};
  int w = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    int face = -1;
    if (c[a] < 0)
      face = 2 * a;
    else if (c[a] >= n[a])
      face = 2 * a + 1;
    if (face < 0) continue;
    const int b = face_kind(g, face);
    if (b == BND_PERIODIC) {
      c[a] += (face & 1) ? -n[a] : n[a];
    } else {
      int t = (b == BND_NOSLIP) ? T_NOSLIP : T_FREESLIP;
      if (w != T_NOSLIP) w = t;
    }
  }
  *wall = w;
  if (w) return -1;
  return (int64_t)(c[0] + g.nx * (c[1] + g.ny * c[2]));
}

// Index of the point (x,y,z), any distance outside the domain, after periodic
// wrap, or -1 beyond a wall face (*wall as for nb_index).
__device__ __forceinline__ int64_t wrap_index(const Geom& g, int x, int y, int z, int* wall) {
  int c[3] = {x, y, z};
  const int n[3] = {g.nx, g.ny, g.nz};
  int w = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (c[a] >= 0 && c[a] < n[a]) continue;
    const int b = face_kind(g, c[a] < 0 ? 2 * a : 2 * a + 1);
    if (b == BND_PERIODIC) {
      const int m = c[a] % n[a];
      c[a] = m < 0 ? m + n[a] : m;
    } else {
      const int t = (b == BND_NOSLIP) ? T_NOSLIP : T_FREESLIP;
      if (w != T_NOSLIP) w = t;
    }
  }
  *wall = w;
  if (w) return -1;
  return (int64_t)(c[0] + g.nx * (c[1] + g.ny * c[2]));
}

// Type of a neighbour (ghost walls included) and its index (-1 for ghosts).
__device__ __forceinline__ int nb_type(const Geom& g, const uint8_t* flags, int x, int y, int z,
                                       int dx, int dy, int dz, int64_t* idx) {
  int w;
  int64_t j = nb_index(g, x, y, z, dx, dy, dz, &w);
  *idx = j;
  if (j < 0) return w;
  return flags[j] & T_MASK;
}

// Where the population arriving at x in direction k comes from (Sec. 2.1 walls):
// plain neighbour x - c_k; bounce-back at a no-slip obstacle; specular reflection
// at a free-slip obstacle (the axes along which the one-axis step back is an
// obstacle are mirrored; the population leaves y in direction j). A gas source
// (directly or after reflection) is reported as SRC_GAS.
enum { SRC_FLUID = 0, SRC_GAS = 1, SRC_BOUNCE = 2 };

// Mirrored source at a free-slip obstacle: the axes along which the one-axis
// step back from x is an obstacle are mirrored. False when no axis is (a
// diagonal obstacle) or the mirrored point is an obstacle: bounce-back.
// Otherwise *src, *dir (the direction the population leaves *src in) and
// *type (gas or fluid) of the mirrored cell.
template <int Q>
__device__ __forceinline__ bool mirror_source(const Geom& g, const uint8_t* flags, int x, int y, int z, int k,
                                              int64_t* src, int* dir, int* type) {
  const int c[3] = {cxd(k), cyd(k), czd(k)};
  int d[3] = {-c[0], -c[1], -c[2]};
  int cj[3] = {c[0], c[1], c[2]};
  bool any = false;
  for (int a = 0; a < 3; ++a) {
    if (c[a] == 0) continue;
    int e[3] = {0, 0, 0};
    e[a] = -c[a];
    int64_t jj;
    if (is_obst(nb_type(g, flags, x, y, z, e[0], e[1], e[2], &jj))) {
      d[a] += c[a];
      cj[a] = -c[a];
      any = true;
    }
  }
  if (!any) return false;
  int64_t yi;
  const int ty = nb_type(g, flags, x, y, z, d[0], d[1], d[2], &yi);
  if (is_obst(ty)) return false;
  int r = 0;
  for (int i = 0; i < Q; ++i)
    if (cxd(i) == cj[0] && cyd(i) == cj[1] && czd(i) == cj[2]) r = i;
  *src = yi;
  *dir = r;
  *type = ty;
  return true;
}

// Specular part of resolve_source (free-slip source).
template <int Q>
__device__ __forceinline__ int reflect_source(const Geom& g, const uint8_t* flags, int x, int y, int z,
                                           int k, int64_t* src, int* dir) {
  int64_t yi;
  int r, ty;
  if (!mirror_source<Q>(g, flags, x, y, z, k, &yi, &r, &ty)) return SRC_BOUNCE;
  if (ty == T_GAS) return SRC_GAS;
  *src = yi;
  *dir = r;
  return SRC_FLUID;
}

// In-place (AA) layout: the element through which the population arriving at
// cell c = (x, y, z) in direction k streams. A step from an even step count
// reads it there and stores the cell's outgoing population of direction
// opp(k) into it; the step from an odd count finds the arriving population in
// the cell's own entry of plane opp(k). The slot is the plane-k entry of the
// source c - c_k inside the domain (after periodic wrap; gas or fluid), the
// cell's own plane-opp(k) entry where the source is a no-slip wall or
// obstacle (bounce-back), or the mirrored cell's entry at a free-slip one.
// Obstacles are static, so a slot never changes during a run, and the map
// (cell, k) -> slot is one to one, as pull streaming with these walls
// consumes every post-collision population once.
template <int Q>
__device__ __forceinline__ int64_t aa_slot(const Geom& g, const uint8_t* flags, int x, int y, int z,
                                           int64_t c, int k) {
  int w;
  const int64_t j = nb_index(g, x, y, z, -cxd(k), -cyd(k), -czd(k), &w);
  const int st = j >= 0 ? (flags[j] & T_MASK) : w;
  if (!is_obst(st)) return (int64_t)k * g.stride + j;
  if (st == T_FREESLIP) {
    int64_t yi;
    int r, ty;
    if (mirror_source<Q>(g, flags, x, y, z, k, &yi, &r, &ty)) return (int64_t)r * g.stride + yi;
  }
  return (int64_t)opp(k) * g.stride + c;
}

template <int Q>
__device__ __forceinline__ int resolve_source(const Geom& g, const uint8_t* flags, int x, int y,
                                              int z, int k, int64_t* src, int* dir, bool* wall) {
  int64_t j;
  int st = nb_type(g, flags, x, y, z, -cxd(k), -cyd(k), -czd(k), &j);
  *dir = k;
  *src = j;
  *wall = is_obst(st);
  if (st == T_GAS) return SRC_GAS;
  if (is_fluid(st)) return SRC_FLUID;
  if (st == T_NOSLIP) return SRC_BOUNCE;
  return reflect_source<Q>(g, flags, x, y, z, k, src, dir);
}

// ---------------------------------------------------------------------------
// Collision (Sec. 2.1): moments with the half-force shift, second-order
// equilibrium, Guo source, SRT or TRT relaxation. The operation order follows
// the definitions term by term; built without contraction so that every step
// is one rounded IEEE operation.
// ---------------------------------------------------------------------------
template <typename R>
struct CollideParams {
  R omega, omega_m;  // 1/tau and the TRT antisymmetric rate
  R gx, gy, gz;
  R tau0, lambda, cs;  // Smagorinsky model (cs > 0): tau0, TRT magic parameter, C_S
};

// Smagorinsky model (Sec. 2.1): total relaxation time tau0 + tau_t from the
// non-equilibrium momentum flux, tau_t = (sqrt(tau0^2 + 2 sqrt(2) C_S^2 Qbar /
// (rho c_s^4)) - tau0) / 2, Qbar = sqrt(2 Q_ab Q_ab) (sum over all a, b).
template <typename R>
__device__ __forceinline__ R les_tau(R tau0, R cs, R rho, R qxx, R qyy, R qzz, R qxy, R qxz,
                                     R qyz) {
  R s2 = qxx * qxx;
  s2 += qxy * qxy;
  s2 += qxz * qxz;
  s2 += qxy * qxy;
  s2 += qyy * qyy;
  s2 += qyz * qyz;
  s2 += qxz * qxz;
  s2 += qyz * qyz;
  s2 += qzz * qzz;
  const R Qbar = sqrt(R(2) * s2);
  const R cs4 = R(1.0 / 9.0);
  const R tt = R(0.5) * (sqrt(tau0 * tau0 + R(2) * sqrt(R(2)) * cs * cs * Qbar / (rho * cs4)) - tau0);
  return tau0 + tt;
}

template <typename R, int Q, bool SH>
__device__ __forceinline__ void moments(const R* f, R gx, R gy, R gz, R& rho, R& dr, R& ux, R& uy,
                                        R& uz) {
  R r = R(0), j0 = R(0), j1 = R(0), j2 = R(0);
#pragma unroll
  for (int k = 0; k < Q; ++k) r += f[k];
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    if (cxd(k) > 0) j0 += f[k];
    if (cxd(k) < 0) j0 += -f[k];
    if (cyd(k) > 0) j1 += f[k];
    if (cyd(k) < 0) j1 += -f[k];
    if (czd(k) > 0) j2 += f[k];
    if (czd(k) < 0) j2 += -f[k];
  }
  // shifted values: sum h = rho - 1 (the weights sum to one, their first
  // moment vanishes)
  dr = SH ? r : r - R(1);
  rho = SH ? R(1) + r : r;
  ux = (j0 + R(0.5) * (rho * gx)) / rho;
  uy = (j1 + R(0.5) * (rho * gy)) / rho;
  uz = (j2 + R(0.5) * (rho * gz)) / rho;
}

// Velocity of the collision that produced the post-collision populations fs:
// sum c f* = sum c f + F, so u = (sum c f* - F/2) / rho with rho = sum f*.
template <typename R, int Q, bool SH>
__device__ __forceinline__ void post_moments(const R* fs, R gx, R gy, R gz, R& rho, R& ux, R& uy,
                                             R& uz) {
  R r = R(0), j0 = R(0), j1 = R(0), j2 = R(0);
#pragma unroll
  for (int k = 0; k < Q; ++k) r += fs[k];
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    if (cxd(k) > 0) j0 += fs[k];
    if (cxd(k) < 0) j0 += -fs[k];
    if (cyd(k) > 0) j1 += fs[k];
    if (cyd(k) < 0) j1 += -fs[k];
    if (czd(k) > 0) j2 += fs[k];
    if (czd(k) < 0) j2 += -fs[k];
  }
  rho = SH ? R(1) + r : r;
  ux = (j0 - R(0.5) * (rho * gx)) / rho;
  uy = (j1 - R(0.5) * (rho * gy)) / rho;
  uz = (j2 - R(0.5) * (rho * gz)) / rho;
}

// rho = sum of the populations in binary64 (mass bookkeeping).
template <typename R, int Q, bool SH>
__device__ __forceinline__ double density64(const R* f) {
  double r = 0.0;
#pragma unroll
  for (int k = 0; k < Q; ++k) r += (double)f[k];
  return SH ? 1.0 + r : r;
}

template <typename R>
__device__ __forceinline__ R cdot(int cx, int cy, int cz, R ax, R ay, R az) {
  // c.a for c in {-1,0,1}^3 without multiplications (exact)
  R s = R(0);
  if (cx > 0) s += ax;
  if (cx < 0) s += -ax;
  if (cy > 0) s += ay;
  if (cy < 0) s += -ay;
  if (cz > 0) s += az;
  if (cz < 0) s += -az;
  return s;
}

// Equilibrium (Sec. 2.1) of direction k; shifted: feq_k - w_k, written with
// dr = rho - 1 so that no large term cancels.
template <typename R, int Q, bool SH>
__device__ __forceinline__ R feq_k(int k, R rho, R dr, R cu, R usq) {
  if (SH) return R(weight<Q>(k)) * (dr + rho * (R(3) * cu + R(4.5) * cu * cu - R(1.5) * usq));
  return R(weight<Q>(k)) * rho * (R(1) + R(3) * cu + R(4.5) * cu * cu - R(1.5) * usq);
}

// f <- collide(f); returns pre-collision rho and u (u with the half-force shift).
// The shift commutes with the relaxation (f - feq = h - heq) and the source sums
// to zero, so the same update applies to f and to h.
template <typename R, int Q, bool TRT, bool SH>
__device__ __forceinline__ void collide(R* f, const CollideParams<R>& cp, R& rho, R& ux, R& uy,
                                        R& uz) {
  R dr;
  moments<R, Q, SH>(f, cp.gx, cp.gy, cp.gz, rho, dr, ux, uy, uz);
  const R Fx = rho * cp.gx, Fy = rho * cp.gy, Fz = rho * cp.gz;
  const R usq = ux * ux + uy * uy + uz * uz;
  R fe[Q], S[Q];
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    const R cu = cdot<R>(cxd(k), cyd(k), czd(k), ux, uy, uz);
    const R cF = cdot<R>(cxd(k), cyd(k), czd(k), Fx, Fy, Fz);
    const R cmuF = (R(cxd(k)) - ux) * Fx + (R(cyd(k)) - uy) * Fy + (R(czd(k)) - uz) * Fz;
    fe[k] = feq_k<R, Q, SH>(k, rho, dr, cu, usq);
    S[k] = R(weight<Q>(k)) * (R(3) * cmuF + R(9) * cu * cF);
  }
  R om = cp.omega, omm = cp.omega_m;
  if (cp.cs > R(0)) {
    // momentum flux of the non-equilibrium part, summed in direction order
    R qxx = R(0), qyy = R(0), qzz = R(0), qxy = R(0), qxz = R(0), qyz = R(0);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const R nq = f[k] - fe[k];
      if (cxd(k) != 0) qxx += nq;
      if (cyd(k) != 0) qyy += nq;
      if (czd(k) != 0) qzz += nq;
      if (cxd(k) * cyd(k) > 0) qxy += nq;
      if (cxd(k) * cyd(k) < 0) qxy += -nq;
      if (cxd(k) * czd(k) > 0) qxz += nq;
      if (cxd(k) * czd(k) < 0) qxz += -nq;
      if (cyd(k) * czd(k) > 0) qyz += nq;
      if (cyd(k) * czd(k) < 0) qyz += -nq;
    }
    const R tau = les_tau<R>(cp.tau0, cp.cs, rho, qxx, qyy, qzz, qxy, qxz, qyz);
    om = R(1) / tau;
    omm = TRT ? R(1) / (R(0.5) + cp.lambda / (tau - R(0.5))) : om;
  }
  if (!TRT) {
    const R sf = R(1) - R(0.5) * om;
#pragma unroll
    for (int k = 0; k < Q; ++k) f[k] = f[k] - om * (f[k] - fe[k]) + sf * S[k];
    return;
  }
  const R sp = R(1) - R(0.5) * om, sm = R(1) - R(0.5) * omm;
  R out[Q];
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    const int kb = opp(k);
    const R fp = R(0.5) * (f[k] + f[kb]), fm = R(0.5) * (f[k] - f[kb]);
    const R ep = R(0.5) * (fe[k] + fe[kb]), em = R(0.5) * (fe[k] - fe[kb]);
    const R p = R(0.5) * (S[k] + S[kb]), m = R(0.5) * (S[k] - S[kb]);
    out[k] = f[k] - om * (fp - ep) - omm * (fm - em) + sp * p + sm * m;
  }
#pragma unroll
  for (int k = 0; k < Q; ++k) f[k] = out[k];
}

// The same collision for the shifted binary32 formats, organised by opposite
// pairs (k, kbar): the symmetric and antisymmetric equilibrium and source parts
// of a pair are formed once,
//   e+ = w (dr + rho (4.5 (c.u)^2 - 1.5 u^2)),  e- = 3 w rho (c.u),
//   S+ = w (9 (c.u)(c.F) - 3 u.F),              S- = 3 w (c.F),
// and f*_k = f_k + n+ + n-, f*_kbar = f_kbar + n+ - n- with
// n+- = -omega+- (f+- - e+-) + (1 - omega+-/2) S+-. SRT is omega- = omega+.
// Algebraically identical to collide(); about half the arithmetic.
template <int Q, bool TRT>
__device__ __forceinline__ void collide_pairs(float* f, const CollideParams<float>& cp, float& rho,
                                              float& ux, float& uy, float& uz) {
  float r = 0.f, j0 = 0.f, j1 = 0.f, j2 = 0.f;
#pragma unroll
  for (int k = 0; k < Q; ++k) r += f[k];
#pragma unroll
  for (int k = 1; k < Q; k += 2) {
    const float d = f[k] - f[k + 1];  // c_k f_k + c_kbar f_kbar = c_k (f_k - f_kbar)
    if (cxd(k) > 0) j0 += d;
    if (cxd(k) < 0) j0 -= d;
    if (cyd(k) > 0) j1 += d;
    if (cyd(k) < 0) j1 -= d;
    if (czd(k) > 0) j2 += d;
    if (czd(k) < 0) j2 -= d;
  }
  const float dr = r;
  rho = 1.f + r;
  const float inv = 1.f / rho;
  ux = (j0 + 0.5f * (rho * cp.gx)) * inv;
  uy = (j1 + 0.5f * (rho * cp.gy)) * inv;
  uz = (j2 + 0.5f * (rho * cp.gz)) * inv;
  const float Fx = rho * cp.gx, Fy = rho * cp.gy, Fz = rho * cp.gz;
  const float usq = ux * ux + uy * uy + uz * uz;
  const float uF = ux * Fx + uy * Fy + uz * Fz;
  float om = cp.omega, omm = TRT ? cp.omega_m : cp.omega;
  if (cp.cs > 0.f) {
    // non-equilibrium momentum flux: each pair contributes c_a c_b 2 (f+ - e+)
    float qxx = 0.f, qyy = 0.f, qzz = 0.f, qxy = 0.f, qxz = 0.f, qyz = 0.f;
#pragma unroll
    for (int k = 1; k < Q; k += 2) {
      const float cu = cdot<float>(cxd(k), cyd(k), czd(k), ux, uy, uz);
      const float ep = float(weight<Q>(k)) * (dr + rho * (4.5f * cu * cu - 1.5f * usq));
      const float nq = (f[k] + f[k + 1]) - 2.f * ep;
      if (cxd(k) != 0) qxx += nq;
      if (cyd(k) != 0) qyy += nq;
      if (czd(k) != 0) qzz += nq;
      if (cxd(k) * cyd(k) > 0) qxy += nq;
      if (cxd(k) * cyd(k) < 0) qxy -= nq;
      if (cxd(k) * czd(k) > 0) qxz += nq;
      if (cxd(k) * czd(k) < 0) qxz -= nq;
      if (cyd(k) * czd(k) > 0) qyz += nq;
      if (cyd(k) * czd(k) < 0) qyz -= nq;
    }
    const float tau = les_tau<float>(cp.tau0, cp.cs, rho, qxx, qyy, qzz, qxy, qxz, qyz);
    om = 1.f / tau;
    omm = TRT ? 1.f / (0.5f + cp.lambda / (tau - 0.5f)) : om;
  }
  const float ap = 1.f - 0.5f * om, am = 1.f - 0.5f * omm;
  {
    const float w0 = float(weight<Q>(0));
    const float ep0 = w0 * (dr - rho * 1.5f * usq);
    const float sp0 = w0 * (-3.f * uF);
    f[0] = f[0] - om * (f[0] - ep0) + ap * sp0;
  }
#pragma unroll
  for (int k = 1; k < Q; k += 2) {
    const float w = float(weight<Q>(k));
    const float cu = cdot<float>(cxd(k), cyd(k), czd(k), ux, uy, uz);
    const float cF = cdot<float>(cxd(k), cyd(k), czd(k), Fx, Fy, Fz);
    const float ep = w * (dr + rho * (4.5f * cu * cu - 1.5f * usq));
    const float em = w * (3.f * rho * cu);
    const float sp = w * (9.f * cu * cF - 3.f * uF);
    const float sm = w * (3.f * cF);
    const float fp = 0.5f * (f[k] + f[k + 1]), fm = 0.5f * (f[k] - f[k + 1]);
    const float np = -om * (fp - ep) + ap * sp;
    const float nm = -omm * (fm - em) + am * sm;
    f[k] = f[k] + np + nm;
    f[k + 1] = f[k + 1] + np - nm;
  }
}

// Collision dispatch: the binary64 path keeps the term-by-term form above;
// the shifted binary32 formats use the pair form.
template <typename R, int Q, bool TRT, bool SH>
__device__ __forceinline__ void collide_any(R* f, const CollideParams<R>& cp, R& rho, R& ux, R& uy,
                                            R& uz) {
  if constexpr (SH && sizeof(R) == 4)
    collide_pairs<Q, TRT>(f, cp, rho, ux, uy, uz);
  else
    collide<R, Q, TRT, SH>(f, cp, rho, ux, uy, uz);
}

// Anti-bounce-back value (Sec. 2.2): feq_k + feq_kbar at (rhoG, u) minus the
// cell's own post-collision f*_kbar; the odd parts cancel. Shifted:
// h_k = 2 w_k (rhoG - 1 + rhoG (4.5 (c.u)^2 - 1.5 u^2)) - h*_kbar.
template <typename R, int Q, bool SH>
__device__ __forceinline__ R abb_value(int k, R rhoG, R ux, R uy, R uz, R usq, R fs_kbar) {
  const R cu = cdot<R>(cxd(k), cyd(k), czd(k), ux, uy, uz);
  if (SH)
    return R(2) * R(weight<Q>(k)) * ((rhoG - R(1)) + rhoG * (R(4.5) * cu * cu - R(1.5) * usq)) -
           fs_kbar;
  return R(2) * R(weight<Q>(k)) * rhoG * (R(1) + R(4.5) * cu * cu - R(1.5) * usq) - fs_kbar;
}

}  // namespace fslbm
