// HIP kernels of the free-surface LBM step for gfx950.
//
// One time step is three launches (plus two for surface tension, two for the
// bubble volume); the last two do their work only when some cell was marked:
//   k_stream    three roles       : every liquid cell away from walls (chunk
//                                   list; pull streaming, collision - the
//                                   bandwidth part), every liquid cell next to
//                                   a wall or obstacle, and every interface cell
//                                   of the compacted list (streaming, free-
//                                   surface condition with the variant's set,
//                                   mass exchange, fill level, conversion mark,
//                                   collision)
//   k_retype    mark-list-driven  : new types around every marked cell (to-gas
//                                   marks next to a to-liquid mark are dropped);
//                                   lists of the new interface cells
//   k_compact   every cell        : the new interface, converted, liquid-chunk
//                                   and wall-liquid lists, compacted in ascending
//                                   order by a single-pass scan (block scan +
//                                   published tile counts); beside it, worker
//                                   blocks complete the conversion: converted
//                                   cells, reinitialisation of the new interface
//                                   cells from gas, and the excess-mass gather,
//                                   fill level and flux classes of every
//                                   interface cell next to a changed cell
// The state between steps is the post-collision population f* (grid A); the
// step writes grid B and the host swaps A/B. Marks, counters and lists stay on the
// device, so a step needs no host synchronisation.
#pragma once

#include <type_traits>

#include "fslbm_device.h"

namespace fslbm {

constexpr int kBlock = 256;
constexpr int kMaxTiles = 4096;  // compaction tiles at most (tile size grows with the domain)
constexpr int kCompBlock = 1024;  // threads of a compaction block

struct Dev {
  Geom g;
  // parameters
  double omega, omega_m, gx, gy, gz;
  double tau0, lambda, cs;  // Smagorinsky model (cs = 0: off)
  double sigma, eps, delta;
  int variant, thurey, bubble;
  // state
  void* fA;  // post-collision populations at t (read)
  void* fB;  // post-collision populations at t+1 (written); in place (aa): fA
  int aa;    // 1: one grid updated in place (AA pattern), slots as aa_slot
  int32_t stash_cap;  // in place: entries of one stash buffer
  // in place: two stash buffers (by step parity) of stash_cap entries of q
  // populations: each interface cell's own post-collision populations, which
  // its neighbours overwrite in the grid during the step; prevpos[c] is the
  // entry of cell c in the buffer the step reads
  void* stash;
  int32_t* prevpos;
  uint8_t* flags;
  uint8_t* mark;
  uint8_t* cls;
  double* phiA;  // fill level at t (valid for every cell)
  double* phiB;  // fill level at t+1
  double* m;     // interface mass
  double* rho_if;
  double* rhoG;  // per-cell gas density (surface tension), or null
  double* phis;  // smoothed fill level (surface tension), or null
  int32_t* smap;  // surface tension: per smoothing tile, the step tag of its last use
  double* lost;  // per-cell lost excess mass
  int32_t* if_list;
  int32_t* conv_list;
  int32_t* chunk_list;  // 64-cell chunks with liquid cells, ascending
  uint64_t* chunk_mask;  // per chunk entry: bit l = cell 64 chunk + l is liquid and not COMPLEX
  int32_t* gen_list;    // liquid cells with the BORDER flag, ascending
  int32_t* mark_list;   // cells marked in this step (unordered)
  int32_t* ng_list;     // new interface cells from gas of this step (unordered)
  int32_t* nl_list;     // new interface cells from liquid of this step (unordered)
  int32_t* cnt;
  unsigned long long* scan_status;  // two words per compaction tile
  double* pV;  // device scalars: [0] p^V, [1] p^V(0), [2] V(0)
  // tracked bubbles (bubble model 2), N each, or null: label per cell (-1:
  // no bubble) and the new labels while they are found; at a bubble's label
  // index its volume, its former cells' volume, the amount handed to it, its
  // amount and pressure, and whether any old bubble handed it an amount
  int32_t* blab;
  int32_t* bpar;
  int32_t* btgt;  // at an old bubble's label: the smallest new label among its cells
  // (the sums bV, bW, bR, bnn as order-free totals: integer part, fraction
  // times 2^64; fix_value reads them)
  int64_t *bV, *bW, *bR, *bnn;
  uint64_t *bVl, *bWl, *bRl, *bnnl;
  double *bamt, *bpr;
  uint8_t* bhas;
  double* partial;  // reduction partials
  int64_t step;  // parity selects the mark-counter slot
};

// Entries of the interface list: the cell index, with bit 31 set when the
// cell has the BORDER bit (its neighbourhood needs wall/wrap handling).
__device__ __forceinline__ int32_t list_entry(int64_t c, bool border) {
  return (int32_t)((uint32_t)c | (border ? 0x80000000u : 0u));
}
__device__ __forceinline__ int64_t list_cell(int32_t e) { return (int64_t)((uint32_t)e & 0x7fffffffu); }
__device__ __forceinline__ bool list_border(int32_t e) { return e < 0; }

// ---------------------------------------------------------------------------
// k_liquid and k_generic
// ---------------------------------------------------------------------------
template <int S, int Q>
__device__ __forceinline__ void load_plain(const typename Store<S, Q>::T* A, int64_t stride,
                                           int64_t c, int nx, int64_t nxy,
                                           typename Store<S, Q>::R* f) {
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    const int64_t off = cxd(k) + (int64_t)cyd(k) * nx + (int64_t)czd(k) * nxy;
    f[k] = Store<S, Q>::ld(A, k * stride + c - off, k);
  }
}

template <typename R>
__device__ __forceinline__ bool unstable(R rho, R ux, R uy, R uz) {
  const R usq = ux * ux + uy * uy + uz * uz;
  return !(rho > R(0)) || !(usq < R(1.0 / 3.0)) || !(rho == rho) || !(usq == usq) ||
         rho > R(1e30);
}

// Liquid cell without the COMPLEX flag: pull from the linear neighbour
// offsets, or - for a cell on a no-slip domain face - bounce-back of its own
// opposite population where the source lies beyond the face; collision; store.
// (A liquid cell never has a gas neighbour, so no free-surface logic applies.)
// BUF: both grids fit a 32-bit byte range, so loads and stores go through
// buffer resources; inside the domain a wave uses one per-lane offset (the
// cell) plus a scalar offset per direction (plane start minus the neighbour
// offset).
// `mine`: the cell is liquid and not COMPLEX (its chunk entry's mask bit).
// Such a cell has no obstacle in its 3x3x3 box and meets only no-slip domain
// faces, so it has the BORDER bit exactly when it lies on a domain face.
template <int S, int Q, bool TRT, bool BUF>
__device__ __forceinline__ void liquid_cell(const Dev& d, int64_t c, bool mine) {
  using St = Store<S, Q>;
  using T = typename St::T;
  using R = typename St::R;
  const Geom& g = d.g;
  bool wall = false;
  if (mine) {
    int x, y, z;
    coords(g, c, x, y, z);
    wall = x == 0 || y == 0 || z == 0 || x == g.nx - 1 || y == g.ny - 1 || z == g.nz - 1;
  }
  const bool any_wall = __ballot(wall) != 0ull;
  if (!mine) return;
  const T* A = static_cast<const T*>(d.fA);
  T* B = static_cast<T*>(d.fB);
  const int64_t stride = g.stride;
  const int64_t nx = g.nx, nxy = (int64_t)g.nx * g.ny;
  R f[Q];
  if (any_wall) {
    // some lane of the wave sits on a no-slip face: per-lane source offsets
    int x, y, z;
    coords(g, c, x, y, z);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const int64_t off = cxd(k) + cyd(k) * nx + czd(k) * nxy;
      const bool in = (unsigned)(x - cxd(k)) < (unsigned)g.nx &&
                      (unsigned)(y - cyd(k)) < (unsigned)g.ny &&
                      (unsigned)(z - czd(k)) < (unsigned)g.nz;
      const int64_t e = in ? k * stride + c - off : opp(k) * stride + c;
      if constexpr (BUF) {
        const __amdgpu_buffer_rsrc_t ra =
            make_rsrc(A, (uint32_t)(Q * stride * (int64_t)sizeof(T)));
        f[k] = St::bld(ra, (uint32_t)(e * (int64_t)sizeof(T)), 0u);
      } else {
        f[k] = St::ld(A, e, in ? k : opp(k));
      }
    }
  } else if constexpr (BUF) {
    const uint32_t bytes = (uint32_t)(Q * stride * (int64_t)sizeof(T));
    const __amdgpu_buffer_rsrc_t ra = make_rsrc(A, bytes);
    const uint32_t vo = (uint32_t)c * (uint32_t)sizeof(T);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const int64_t off = cxd(k) + cyd(k) * nx + czd(k) * nxy;
      f[k] = St::bld(ra, vo, (uint32_t)((k * stride - off) * (int64_t)sizeof(T)));
    }
  } else {
    load_plain<S, Q>(A, stride, c, g.nx, nxy, f);
  }
  CollideParams<R> cp{R(d.omega), R(d.omega_m), R(d.gx), R(d.gy), R(d.gz), R(d.tau0), R(d.lambda), R(d.cs)};
  R rho, ux, uy, uz;
  collide_any<R, Q, TRT, St::kShift>(f, cp, rho, ux, uy, uz);
  if (unstable(rho, ux, uy, uz)) atomicOr(&d.cnt[CNT_ERR], ERR_UNSTABLE);
  if constexpr (BUF) {
    const uint32_t bytes = (uint32_t)(Q * stride * (int64_t)sizeof(T));
    const __amdgpu_buffer_rsrc_t rb = make_rsrc(B, bytes);
    const uint32_t vo = (uint32_t)c * (uint32_t)sizeof(T);
#pragma unroll
    for (int k = 0; k < Q; ++k) St::bst(rb, vo, (uint32_t)(k * stride * (int64_t)sizeof(T)), f[k]);
  } else {
#pragma unroll
    for (int k = 0; k < Q; ++k) St::st(B, k * stride + c, k, f[k]);
  }
}

// In-place layout: element of the post-collision population f*_k(c) of the
// state before a step of parity `par` (cell c with flag byte fl): plane k of c
// after an odd step (or at the start), else the slot through which the cell's
// arrival from direction opp(k) streamed, where the even step stored it (for
// a cell without the BORDER bit, plane opp(k) of its neighbour c + c_k).
template <int Q>
__device__ __forceinline__ int64_t own_slot(const Dev& d, int64_t c, uint8_t fl, int k, int par) {
  const int64_t stride = d.g.stride;
  if (!d.aa || par == 0) return (int64_t)k * stride + c;
  if (!(fl & F_BORDER))
    return (int64_t)opp(k) * stride + c + cxd(k) + cyd(k) * (int64_t)d.g.nx + czd(k) * (int64_t)d.g.nx * d.g.ny;
  int x, y, z;
  coords(d.g, c, x, y, z);
  return aa_slot<Q>(d.g, d.flags, x, y, z, c, opp(k));
}

// In-place layout: entry e of the stash buffer of step parity par.
template <int S, int Q>
__device__ __forceinline__ typename Store<S, Q>::T* stash_buf(const Dev& d, int par) {
  return static_cast<typename Store<S, Q>::T*>(d.stash) + (int64_t)par * d.stash_cap * Q;
}

// liquid_cell in the in-place layout. Even step: the arrival from direction
// k is read from its slot (the pull source, or the cell's own opposite
// population on a no-slip face), and the outgoing population of direction
// opp(k) is stored into that slot after the collision. Odd step: arrivals are
// the cell's own plane-opp(k) entries, outgoing populations go to its own
// plane-k entries (walls were handled by the even step's placement).
template <int S, int Q, bool TRT, bool BUF>
__device__ __forceinline__ void liquid_cell_aa(const Dev& d, int64_t c, bool mine) {
  using St = Store<S, Q>;
  using T = typename St::T;
  using R = typename St::R;
  const Geom& g = d.g;
  const bool odd = (d.step & 1) != 0;
  bool wall = false;
  if (mine && !odd) {
    int x, y, z;
    coords(g, c, x, y, z);
    wall = x == 0 || y == 0 || z == 0 || x == g.nx - 1 || y == g.ny - 1 || z == g.nz - 1;
  }
  const bool any_wall = !odd && __ballot(wall) != 0ull;
  if (!mine) return;
  T* F = static_cast<T*>(d.fA);
  const int64_t stride = g.stride;
  const int64_t nx = g.nx, nxy = (int64_t)g.nx * g.ny;
  const uint32_t bytes = (uint32_t)(BUF ? Q * stride * (int64_t)sizeof(T) : 0);
  const uint32_t vo = (uint32_t)c * (uint32_t)sizeof(T);
  R f[Q];
  if (odd) {
    // own entries only: arrival k in plane opp(k)
    if constexpr (BUF) {
      const __amdgpu_buffer_rsrc_t ra = make_rsrc(F, bytes);
#pragma unroll
      for (int k = 0; k < Q; ++k) f[k] = St::bld(ra, vo, (uint32_t)(opp(k) * stride * (int64_t)sizeof(T)));
    } else {
#pragma unroll
      for (int k = 0; k < Q; ++k) f[k] = St::ld(F, opp(k) * stride + c, k);
    }
  } else if (!any_wall) {
    // the pull sources, as the two-grid liquid cell
    if constexpr (BUF) {
      const __amdgpu_buffer_rsrc_t ra = make_rsrc(F, bytes);
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        const int64_t off = cxd(k) + cyd(k) * nx + czd(k) * nxy;
        f[k] = St::bld(ra, vo, (uint32_t)((k * stride - off) * (int64_t)sizeof(T)));
      }
    } else {
      load_plain<S, Q>(F, stride, c, g.nx, nxy, f);
    }
  } else {
    int x, y, z;
    coords(g, c, x, y, z);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const int64_t off = cxd(k) + cyd(k) * nx + czd(k) * nxy;
      const bool in = (unsigned)(x - cxd(k)) < (unsigned)g.nx && (unsigned)(y - cyd(k)) < (unsigned)g.ny &&
                      (unsigned)(z - czd(k)) < (unsigned)g.nz;
      f[k] = St::ld(F, in ? k * stride + c - off : opp(k) * stride + c, k);
    }
  }
  CollideParams<R> cp{R(d.omega), R(d.omega_m), R(d.gx), R(d.gy), R(d.gz), R(d.tau0), R(d.lambda), R(d.cs)};
  R rho, ux, uy, uz;
  collide_any<R, Q, TRT, St::kShift>(f, cp, rho, ux, uy, uz);
  if (unstable(rho, ux, uy, uz)) atomicOr(&d.cnt[CNT_ERR], ERR_UNSTABLE);
  if (odd) {
    if constexpr (BUF) {
      const __amdgpu_buffer_rsrc_t rb = make_rsrc(F, bytes);
#pragma unroll
      for (int k = 0; k < Q; ++k) St::bst(rb, vo, (uint32_t)(k * stride * (int64_t)sizeof(T)), f[k]);
    } else {
#pragma unroll
      for (int k = 0; k < Q; ++k) St::st(F, k * stride + c, k, f[k]);
    }
  } else if (!any_wall) {
    // outgoing opp(k) into the slot arrival k came from
    if constexpr (BUF) {
      const __amdgpu_buffer_rsrc_t rb = make_rsrc(F, bytes);
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        const int64_t off = cxd(k) + cyd(k) * nx + czd(k) * nxy;
        St::bst(rb, vo, (uint32_t)((k * stride - off) * (int64_t)sizeof(T)), f[opp(k)]);
      }
    } else {
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        const int64_t off = cxd(k) + cyd(k) * nx + czd(k) * nxy;
        St::st(F, k * stride + c - off, k, f[opp(k)]);
      }
    }
  } else {
    int x, y, z;
    coords(g, c, x, y, z);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const int64_t off = cxd(k) + cyd(k) * nx + czd(k) * nxy;
      const bool in = (unsigned)(x - cxd(k)) < (unsigned)g.nx && (unsigned)(y - cyd(k)) < (unsigned)g.ny &&
                      (unsigned)(z - czd(k)) < (unsigned)g.nz;
      St::st(F, in ? k * stride + c - off : opp(k) * stride + c, k, f[opp(k)]);
    }
  }
}

// Mass-flux term between interface cells with the forced fill/empty rule:
// equal classes exchange in - out; a cell that should fill only receives, one
// that should empty only gives. Antisymmetric, so mass is conserved.
__device__ __forceinline__ double flux_term(int cx, int cn, double in, double out) {
  if (cx == cn) return in - out;
  if (cn == CLS_NOLIQ) return in;
  if (cx == CLS_NOGAS && cn == CLS_STD) return in;
  return -out;
}

// ---------------------------------------------------------------------------
// List-driven kernels work on one cell per group of 32 lanes: lane k handles
// lattice direction k (lanes >= q idle in the direction work). Sums over
// directions are butterfly reductions over the group: every lane performs the
// same additions (a + b and b + a round alike), so all lanes hold the same,
// deterministic result. The order differs from a sequential loop only by
// rounding.
// ---------------------------------------------------------------------------
constexpr int kG = 32;

// Lane exchanges inside a 32-lane group on 32-bit words: DPP row operations
// (xor 1 and xor 2 within a quad, mirror within 8 and within 16 lanes) and
// one swizzle (xor 16). After the four row steps of a sum every lane of a
// 16-lane row holds the row sum; the swizzle adds the other row of the group.
template <int CTRL>
__device__ __forceinline__ int dpp32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, true);
}
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;  // lane i <-> 7 - i within 8
constexpr int kDppMirror = 0x140;      // lane i <-> 15 - i within 16
constexpr int kSwzXor16 = 0x401F;      // bitmask mode: and 0x1f, xor 0x10

template <int CTRL>
__device__ __forceinline__ float dppf(float v) {
  return __int_as_float(dpp32<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ double dppd(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp32<CTRL>((int)b), hi = dpp32<CTRL>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float swz16f(float v) {
  return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), kSwzXor16));
}
__device__ __forceinline__ double swz16d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_swizzle((int)b, kSwzXor16);
  const int hi = __builtin_amdgcn_ds_swizzle((int)(b >> 32), kSwzXor16);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 32 lanes of the group (callers pass 0 from lanes that do not
// take part). Each step adds a lane's value to its partner's in the same
// order on both sides (a + b and b + a round alike), so every lane ends with
// the same, deterministic sum; it differs from a sequential sum only by
// rounding.
__device__ __forceinline__ float gsum(float v, int) {
  v += dppf<kDppXor1>(v);
  v += dppf<kDppXor2>(v);
  v += dppf<kDppHalfMirror>(v);
  v += dppf<kDppMirror>(v);
  return v + swz16f(v);
}
__device__ __forceinline__ double gsum(double v, int) {
  v += dppd<kDppXor1>(v);
  v += dppd<kDppXor2>(v);
  v += dppd<kDppHalfMirror>(v);
  v += dppd<kDppMirror>(v);
  return v + swz16d(v);
}

// ballot restricted to the calling lane's group (bit k = lane k of the group)
__device__ __forceinline__ uint32_t gballot(bool p) {
  return (uint32_t)(__ballot(p) >> (threadIdx.x & 32));
}

// Work items [0, n) of a role split over the XCDs: consecutive blocks of a
// launch run on consecutive XCDs (round robin), each with its own L2, so
// block blk (blk mod kXcds is its XCD when the role starts at a multiple of
// kXcds) takes a slice of a contiguous range of the items: neighbouring cells,
// whose populations share cache lines, are processed under one L2.
constexpr int kXcds = 8;
struct XcdRange {
  int begin, end, first, step;  // items [begin, end), this unit's first item and stride
};
__device__ __forceinline__ XcdRange xcd_range(int n, int blk, int nblk, int unit, int units_per_block) {
  const int x = blk % kXcds;
  const int blocks_x = (nblk - x + kXcds - 1) / kXcds;  // blocks of this role on XCD x
  const int r = blk / kXcds;
  XcdRange q;
  q.begin = (int)((int64_t)n * x / kXcds);
  q.end = (int)((int64_t)n * (x + 1) / kXcds);
  q.first = q.begin + r * units_per_block + unit;
  q.step = blocks_x * units_per_block;
  return q;
}

// Collision of one cell held one direction per lane (f = population of this
// lane's direction k); same arithmetic as collide().
template <typename R, int Q, bool TRT, bool SH>
__device__ __forceinline__ R gcollide(R f, int k, const CollideParams<R>& cp, R& rho, R& ux, R& uy,
                                      R& uz) {
  const bool act = k < Q;
  const int kk = act ? k : 0;
  const int cx = cxd(kk), cy = cyd(kk), cz = czd(kk);
  const R fv = act ? f : R(0);
  const R r = gsum(fv, Q);
  const R j0 = gsum(cx > 0 ? fv : (cx < 0 ? -fv : R(0)), Q);
  const R j1 = gsum(cy > 0 ? fv : (cy < 0 ? -fv : R(0)), Q);
  const R j2 = gsum(cz > 0 ? fv : (cz < 0 ? -fv : R(0)), Q);
  const R dr = SH ? r : r - R(1);
  rho = SH ? R(1) + r : r;
  ux = (j0 + R(0.5) * (rho * cp.gx)) / rho;
  uy = (j1 + R(0.5) * (rho * cp.gy)) / rho;
  uz = (j2 + R(0.5) * (rho * cp.gz)) / rho;
  const R Fx = rho * cp.gx, Fy = rho * cp.gy, Fz = rho * cp.gz;
  const R usq = ux * ux + uy * uy + uz * uz;
  const R cu = cdot<R>(cx, cy, cz, ux, uy, uz);
  const R cF = cdot<R>(cx, cy, cz, Fx, Fy, Fz);
  const R cmuF = (R(cx) - ux) * Fx + (R(cy) - uy) * Fy + (R(cz) - uz) * Fz;
  const R w = R(weight<Q>(kk));
  const R fe = SH ? w * (dr + rho * (R(3) * cu + R(4.5) * cu * cu - R(1.5) * usq))
                  : w * rho * (R(1) + R(3) * cu + R(4.5) * cu * cu - R(1.5) * usq);
  const R S = w * (R(3) * cmuF + R(9) * cu * cF);
  R om = cp.omega, omm = cp.omega_m;
  if (cp.cs > R(0)) {
    const R nq = act ? fv - fe : R(0);
    const R qxx = gsum(cx != 0 ? nq : R(0), Q), qyy = gsum(cy != 0 ? nq : R(0), Q);
    const R qzz = gsum(cz != 0 ? nq : R(0), Q);
    const R qxy = gsum(R(cx * cy) * nq, Q), qxz = gsum(R(cx * cz) * nq, Q);
    const R qyz = gsum(R(cy * cz) * nq, Q);
    const R tau = les_tau<R>(cp.tau0, cp.cs, rho, qxx, qyy, qzz, qxy, qxz, qyz);
    om = R(1) / tau;
    omm = TRT ? R(1) / (R(0.5) + cp.lambda / (tau - R(0.5))) : om;
  }
  if (!TRT) return fv - om * (fv - fe) + (R(1) - R(0.5) * om) * S;
  const int kb = opp(kk);
  const R fb = __shfl(fv, kb, kG), eb = __shfl(fe, kb, kG), Sb = __shfl(S, kb, kG);
  const R fp = R(0.5) * (fv + fb), fm = R(0.5) * (fv - fb);
  const R ep = R(0.5) * (fe + eb), em = R(0.5) * (fe - eb);
  const R p = R(0.5) * (S + Sb), m = R(0.5) * (S - Sb);
  return fv - om * (fp - ep) - omm * (fm - em) + (R(1) - R(0.5) * om) * p +
         (R(1) - R(0.5) * omm) * m;
}

// Interface cells: streaming, free-surface condition, mass exchange, fill
// level, conversion mark, collision. Lane k of the cell's group pulls
// direction k from x - c_k; lanes below 27 also read the 3x3x3 neighbour used
// by the normal. Every load of the cell is issued in one batch (indices of
// neighbours beyond a wall are replaced by the cell itself and the values
// discarded); only a source reflected at a free-slip face needs a second
// round.
// In-place layout, conversion of step `step`: a stash entry of the next
// step's buffer for a new interface cell (after the entries of the cells
// that were interface in this step), recorded in prevpos; -1 (and ERR_STASH)
// when the buffer is full. Lane 0 of the calling group takes it.
__device__ __forceinline__ int32_t new_stash_entry(const Dev& d, int64_t c, int l) {
  int32_t pos = -1;
  if (l == 0) {
    pos = d.cnt[CNT_SBASE] + atomicAdd(&d.cnt[CNT_SNEW], 1);
    if (pos >= d.stash_cap) {
      atomicOr(&d.cnt[CNT_ERR], ERR_STASH);
      pos = -1;
    } else {
      d.prevpos[c] = pos;
    }
  }
  return __shfl(pos, 0, kG);
}

// AA: in-place layout. The cell's own post-collision populations come from
// its stash entry (prevpos) of this step's buffer, written by the previous
// step, since neighbours overwrite them in the grid during this launch; the
// new ones also go to entry `item` of the next step's buffer. An even step
// reads arrivals from their slots as the two-grid pull does and stores the
// outgoing population of direction opp(k) into the slot of lane k; an odd
// step reads arrivals from the cell's own plane-opp(k) entries and stores into
// its own plane-k entries.
template <int S, int Q, bool TRT, bool AA>
__device__ __forceinline__ void generic_role(const Dev& d, int blk, int nblk, int nif) {
  using St = Store<S, Q>;
  using T = typename St::T;
  using R = typename St::R;
  constexpr bool SH = St::kShift;
  const T* A = static_cast<const T*>(d.fA);
  T* B = static_cast<T*>(d.fB);
  const bool odd = AA && (d.step & 1) != 0;
  const Geom& g = d.g;
  const int64_t stride = g.stride;
  const int l = threadIdx.x & (kG - 1);
  const bool act = l < Q;
  const int k = act ? l : 0;
  const int kb = opp(k);
  const int cx = cxd(k), cy = cyd(k), cz = czd(k);
  const int v = d.variant;
  CollideParams<R> cp{R(d.omega), R(d.omega_m), R(d.gx), R(d.gy), R(d.gz), R(d.tau0), R(d.lambda), R(d.cs)};
  // linear offsets of this lane's pull source and box neighbour (cells
  // without the BORDER bit: their whole 3x3x3 box lies inside the domain and
  // holds no obstacle)
  const int64_t gnx = g.nx, gnxy = (int64_t)g.nx * g.ny;
  const int64_t offd = cx + cy * gnx + cz * gnxy;
  const int64_t offb = l < 27 ? (l % 3 - 1) + ((l / 3) % 3 - 1) * gnx + (l / 9 - 1) * gnxy : 0;
  const XcdRange q = xcd_range(nif, blk, nblk, threadIdx.x / kG, kBlock / kG);
  for (int item = q.first; item < q.end; item += q.step) {
    const int32_t e = d.if_list[item];
    const int64_t c = list_cell(e);
    int x = 0, y = 0, z = 0;
    // pull source x - c_k and 3x3x3 neighbour of this lane
    int wd = 0, wb = 0;
    int64_t jd, jb;
    if (list_border(e)) {
      coords(g, c, x, y, z);
      jd = nb_index(g, x, y, z, -cx, -cy, -cz, &wd);
      jb = l < 27 ? nb_index(g, x, y, z, l % 3 - 1, (l / 3) % 3 - 1, l / 9 - 1, &wb) : c;
    } else {
      jd = c - offd;
      jb = c + offb;
    }
    const int64_t js = jd >= 0 ? jd : c, jbs = jb >= 0 ? jb : c;
    // the batch
    R fo, fpull;
    if constexpr (AA) {
      const int32_t pp = d.prevpos[c];
      fo = act ? St::ld(stash_buf<S, Q>(d, (int)(d.step & 1)), (int64_t)pp * Q + k, k) : R(0);
      fpull = act ? St::ld(A, odd ? opp(k) * stride + c : k * stride + js, k) : R(0);
    } else {
      fo = act ? St::ld(A, k * stride + c, k) : R(0);
      fpull = act ? St::ld(A, k * stride + js, k) : R(0);
    }
    const uint8_t flb = d.flags[jbs];
    const double phib = d.phiA[jbs];
    const uint8_t clsb = d.cls[jbs];
    // the cell itself is the box centre (lane 13)
    const uint8_t cls_c = (uint8_t)__shfl((int)clsb, 13, kG);
    const double phi_c = __shfl(phib, 13, kG);
    const double m_c = d.m[c];
    const double rhoG_c = d.rhoG ? d.rhoG[c] : d.pV[0] * 3.0;
    // own post-collision population of the opposite direction
    const R fo_b = __shfl(fo, kb, kG);
    // the pull source x - c_k is the box point of offset -c_k (same index,
    // wrap and ghost), so its flag, fill level and class come from that lane
    const int lb = (1 - cx) + 3 * (1 - cy) + 9 * (1 - cz);
    const uint8_t fld = (uint8_t)__shfl((int)flb, lb, kG);
    const double phid = __shfl(phib, lb, kG);
    const uint8_t clsd = (uint8_t)__shfl((int)clsb, lb, kG);
    // kind of the pull source (Sec. 2.1 walls, Sec. 2.2 gas)
    const int st = jd >= 0 ? (fld & T_MASK) : wd;
    const bool wall = is_obst(st);
    int kind;
    int64_t src = jd;
    int dir = k;
    R in_val = fpull;
    uint8_t fl_src = fld, cls_src = clsd;
    double phi_src = phid;
    if (st == T_GAS) {
      kind = SRC_GAS;
    } else if (is_fluid(st)) {
      kind = SRC_FLUID;
    } else if (st == T_NOSLIP) {
      kind = SRC_BOUNCE;
    } else {
      kind = reflect_source<Q>(g, d.flags, x, y, z, k, &src, &dir);
      if (act && kind == SRC_FLUID) {
        // (in place, odd step: the even step put it into the cell's own entry)
        in_val = odd ? fpull : St::ld(A, dir * stride + src, dir);
        fl_src = d.flags[src];
        cls_src = d.cls[src];
        phi_src = d.phiA[src];
      }
    }
    // velocity of the collision at t, from the post-collision populations
    // (fo is zero on lanes >= q)
    const R r0 = gsum(fo, Q);
    const R a0 = gsum(cx > 0 ? fo : (cx < 0 ? -fo : R(0)), Q);
    const R a1 = gsum(cy > 0 ? fo : (cy < 0 ? -fo : R(0)), Q);
    const R a2 = gsum(cz > 0 ? fo : (cz < 0 ? -fo : R(0)), Q);
    const R rho_t = SH ? R(1) + r0 : r0;
    const R ux = (a0 - R(0.5) * (rho_t * R(d.gx))) / rho_t;
    const R uy = (a1 - R(0.5) * (rho_t * R(d.gy))) / rho_t;
    const R uz = (a2 - R(0.5) * (rho_t * R(d.gz))) / rho_t;
    const R usq = ux * ux + uy * uy + uz * uz;
    // missing populations (direct gas sources) and the variant's set (Sec. 3)
    const uint32_t gas = gballot(act && l > 0 && kind == SRC_GAS && !wall);
    const int missing = __popc(gas);
    const bool nb_based = (v == 1 || v == 2 || (v == 4 && missing < 3));
    bool in_R = ((gas >> k) & 1u) != 0;
    if (nb_based) {
      // Parker-Youngs normal (Sec. 2.2): lane l holds phi at offset
      // (l%3-1, (l/3)%3-1, l/9-1); obstacle points take the centre value
      double vphi = phi_c;
      if (l < 27) {
        const int tb = jb >= 0 ? (flb & T_MASK) : wb;
        vphi = is_obst(tb) ? phi_c : phib;
      }
      // n_a = sum over the box of the lane's Parker-Youngs weight (offset
      // along a times the {1,2,1} weights of the other two offsets) times
      // phi: the terms of the weighted central differences, summed over the
      // group
      double wx = 0.0, wy = 0.0, wz = 0.0;
      if (l < 27) {
        const int ox = l % 3 - 1, oy = (l / 3) % 3 - 1, oz = l / 9 - 1;
        const double Wx = ox == 0 ? 2.0 : 1.0, Wy = oy == 0 ? 2.0 : 1.0, Wz = oz == 0 ? 2.0 : 1.0;
        wx = ox * Wy * Wz;
        wy = oy * Wx * Wz;
        wz = oz * Wx * Wy;
      }
      double n[3];
      n[0] = gsum(wx * vphi, Q);
      n[1] = gsum(wy * vphi, Q);
      n[2] = gsum(wz * vphi, Q);
      double nmax = fabs(n[0]);
      nmax = fabs(n[1]) > nmax ? fabs(n[1]) : nmax;
      nmax = fabs(n[2]) > nmax ? fabs(n[2]) : nmax;
      const double dot = n[0] * cx + n[1] * cy + n[2] * cz;
      if ((k > 0 || v == 1) && dot >= -d.delta * nmax) in_R = true;
    }
    const R rhoG = R(rhoG_c);
    R f;
    if (kind == SRC_BOUNCE)
      f = fo_b;
    else if (kind == SRC_GAS || (in_R && !wall))
      f = abb_value<R, Q, SH>(k, rhoG, ux, uy, uz, usq, fo_b);
    else
      f = in_val;
    // mass exchange (Sec. 2.2) along the actual streaming path of direction k
    double term = 0.0;
    if (act && l > 0 && kind == SRC_FLUID) {
      const double in = (double)in_val, out = (double)fo_b;
      if ((fl_src & T_MASK) == T_LIQ) {
        term = in - out;
      } else {
        const double T_ = d.thurey ? flux_term(cls_c, cls_src, in, out) : in - out;
        term = 0.5 * (phi_c + phi_src) * T_;
      }
    }
    const double dm = gsum(term, Q);
    const double rho_n = (SH ? 1.0 : 0.0) + gsum(act ? (double)f : 0.0, Q);
    const double m_new = m_c + dm;
    const double phi_n = m_new / rho_n;
    uint8_t mk = MK_NONE;
    if (phi_n > 1.0 + d.eps)
      mk = MK_L;
    else if (phi_n < -d.eps)
      mk = MK_G;
    if (l == 0) {
      d.m[c] = m_new;
      d.rho_if[c] = rho_n;
      d.phiB[c] = phi_n;
      d.mark[c] = mk;
      if (mk) d.mark_list[atomicAdd(&d.cnt[CNT_MARK0 + (d.step & 1)], 1)] = (int32_t)c;
      if (!(m_new == m_new)) atomicOr(&d.cnt[CNT_ERR], ERR_UNSTABLE);
      // a new interface cell of the previous conversion loses its transient
      // bits (readers in this kernel look at the type bits only); lane 0
      // pulls the rest direction from the cell itself, so fld is its flag
      const uint8_t fc = fld;
      if (fc & F_TRANSIENT) d.flags[c] = (uint8_t)(fc & ~F_TRANSIENT);
    }
    R rho, vx, vy, vz;
    const R fs = gcollide<R, Q, TRT, SH>(f, l, cp, rho, vx, vy, vz);
    if (l == 0 && unstable(rho, vx, vy, vz)) atomicOr(&d.cnt[CNT_ERR], ERR_UNSTABLE);
    if constexpr (AA) {
      if (act) St::st(stash_buf<S, Q>(d, (int)((d.step + 1) & 1)), (int64_t)item * Q + k, k, fs);
      if (l == 0) d.prevpos[c] = item;
      if (!odd) {
        const R fsb = __shfl(fs, kb, kG);
        const int64_t sl = list_border(e) ? aa_slot<Q>(g, d.flags, x, y, z, c, k) : k * stride + c - offd;
        if (act) St::st(B, sl, k, fsb);
        continue;
      }
    }
    if (act) St::st(B, k * stride + c, k, fs);
  }
}

// Liquid cell with the COMPLEX flag, one thread per cell: each direction's
// source is resolved with periodic wrap, bounce-back at obstacles and specular
// reflection at free-slip faces (a liquid cell never has a gas neighbour).
template <int S, int Q, bool TRT>
__device__ __forceinline__ void border_cell(const Dev& d, int64_t c) {
  using St = Store<S, Q>;
  using T = typename St::T;
  using R = typename St::R;
  const T* A = static_cast<const T*>(d.fA);
  T* B = static_cast<T*>(d.fB);
  const Geom& g = d.g;
  const int64_t stride = g.stride;
  int x, y, z;
  coords(g, c, x, y, z);
  // the pull sources in batches of kBB directions: the batch's types in one
  // load round, then its populations (only a free-slip source needs more
  // reads), so that a cell waits for a few rounds, not two per direction,
  // and only a batch's indices are held at once
  constexpr int kBB = 7;
  R f[Q];
#pragma unroll
  for (int k0 = 0; k0 < Q; k0 += kBB) {
    int64_t jj[kBB];
    int ty[kBB];
#pragma unroll
    for (int i = 0; i < kBB; ++i) {
      const int k = k0 + i;
      if (k >= Q) break;
      int w;
      jj[i] = nb_index(g, x, y, z, -cxd(k), -cyd(k), -czd(k), &w);
      ty[i] = jj[i] >= 0 ? (d.flags[jj[i]] & T_MASK) : w;
    }
#pragma unroll
    for (int i = 0; i < kBB; ++i) {
      const int k = k0 + i;
      if (k >= Q) break;
      int64_t src = jj[i];
      int dir = k;
      const int st = ty[i];
      int kind;
      if (st == T_GAS)
        kind = SRC_GAS;
      else if (is_fluid(st))
        kind = SRC_FLUID;
      else if (st == T_NOSLIP)
        kind = SRC_BOUNCE;
      else
        kind = reflect_source<Q>(g, d.flags, x, y, z, k, &src, &dir);
      if (kind == SRC_GAS) atomicOr(&d.cnt[CNT_ERR], ERR_LAYER);
      if (kind != SRC_FLUID) {
        src = c;
        dir = opp(k);
      }
      f[k] = St::ld(A, dir * stride + src, dir);
    }
  }
  CollideParams<R> cp{R(d.omega), R(d.omega_m), R(d.gx), R(d.gy), R(d.gz), R(d.tau0), R(d.lambda), R(d.cs)};
  R rho, ux, uy, uz;
  collide_any<R, Q, TRT, St::kShift>(f, cp, rho, ux, uy, uz);
  if (unstable(rho, ux, uy, uz)) atomicOr(&d.cnt[CNT_ERR], ERR_UNSTABLE);
#pragma unroll
  for (int k = 0; k < Q; ++k) St::st(B, k * stride + c, k, f[k]);
}

// border_cell in the in-place layout: an even step reads each arrival from
// its slot (for a liquid cell, whose box holds no gas, the resolved source is
// the slot of aa_slot) and stores the outgoing population of the opposite
// direction into it; an odd step uses the cell's own entries only. The even
// step's stores resolve one slot at a time (not unrolled: wall cells are few,
// and unrolled resolution would hold q addresses over the collision and cost
// the whole launch a quarter of its waves).
template <int S, int Q, bool TRT>
__device__ __forceinline__ void border_cell_aa(const Dev& d, int64_t c) {
  using St = Store<S, Q>;
  using T = typename St::T;
  using R = typename St::R;
  T* F = static_cast<T*>(d.fA);
  const Geom& g = d.g;
  const int64_t stride = g.stride;
  const bool odd = (d.step & 1) != 0;
  R f[Q];
  if (odd) {
#pragma unroll
    for (int k = 0; k < Q; ++k) f[k] = St::ld(F, opp(k) * stride + c, k);
  } else {
    int x, y, z;
    coords(g, c, x, y, z);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      int64_t src;
      int dir;
      bool wall;
      const int kind = resolve_source<Q>(g, d.flags, x, y, z, k, &src, &dir, &wall);
      if (kind == SRC_GAS) atomicOr(&d.cnt[CNT_ERR], ERR_LAYER);
      if (kind != SRC_FLUID) {
        src = c;
        dir = opp(k);
      }
      f[k] = St::ld(F, dir * stride + src, dir);
    }
  }
  CollideParams<R> cp{R(d.omega), R(d.omega_m), R(d.gx), R(d.gy), R(d.gz), R(d.tau0), R(d.lambda), R(d.cs)};
  R rho, ux, uy, uz;
  collide_any<R, Q, TRT, St::kShift>(f, cp, rho, ux, uy, uz);
  if (unstable(rho, ux, uy, uz)) atomicOr(&d.cnt[CNT_ERR], ERR_UNSTABLE);
  if (odd) {
#pragma unroll
    for (int k = 0; k < Q; ++k) St::st(F, k * stride + c, k, f[k]);
  } else {
    int x, y, z;
    coords(g, c, x, y, z);
#pragma unroll 1
    for (int k = 0; k < Q; ++k) {
      R v = f[0];
#pragma unroll
      for (int i = 0; i < Q; ++i) v = (opp(k) == i) ? f[i] : v;
      St::st(F, aa_slot<Q>(g, d.flags, x, y, z, c, k), k, v);
    }
  }
}

// Also clears the transient bits of the cells of the last converted list
// (every transient bit is stale by now; readers in this kernel look at the
// type bits only).
template <int S, int Q, bool TRT, bool AA>
__device__ __forceinline__ void border_role(const Dev& d, int blk, int nblk, int n, int ncv) {
  for (int i = blk * kBlock + threadIdx.x; i < n + ncv; i += nblk * kBlock) {
    if (i < n) {
      if constexpr (AA)
        border_cell_aa<S, Q, TRT>(d, d.gen_list[i]);
      else
        border_cell<S, Q, TRT>(d, d.gen_list[i]);
    } else {
      const int32_t z = d.conv_list[i - n];
      d.flags[z] = (uint8_t)(d.flags[z] & ~F_TRANSIENT);
    }
  }
}

// Each wave takes 64-cell chunks from the chunk list (chunks without liquid
// cells are never visited), one cell per lane. The wave's entries (chunk and
// liquid-lane mask) are loaded 64 at a time, one per lane, and read back by
// lane index, so a chunk's population loads wait for no other load.
template <int S, int Q, bool TRT, bool BUF, bool AA>
__device__ __forceinline__ void liquid_role(const Dev& d, int blk, int nblk, int nch) {
  const int lane = threadIdx.x & 63;
  const XcdRange q = xcd_range(nch, blk, nblk, threadIdx.x >> 6, kBlock / 64);
  for (int w0 = q.first; w0 < q.end; w0 += 64 * q.step) {
    const int wl = w0 + lane * q.step;
    const int32_t ch = wl < q.end ? d.chunk_list[wl] : 0;
    const uint64_t mk = wl < q.end ? d.chunk_mask[wl] : 0ull;
    const uint32_t mlo = (uint32_t)mk, mhi = (uint32_t)(mk >> 32);
    for (int it = 0; it < 64 && w0 + it * q.step < q.end; ++it) {
      const int32_t chunk = __builtin_amdgcn_readlane(ch, it);
      const uint32_t half = lane < 32 ? __builtin_amdgcn_readlane(mlo, it) : __builtin_amdgcn_readlane(mhi, it);
      if constexpr (AA)
        liquid_cell_aa<S, Q, TRT, BUF>(d, (int64_t)chunk * 64 + lane, ((half >> (lane & 31)) & 1u) != 0);
      else
        liquid_cell<S, Q, TRT, BUF>(d, (int64_t)chunk * 64 + lane, ((half >> (lane & 31)) & 1u) != 0);
    }
  }
}

// The streaming half of a step in one launch: the three cell classes read
// grid A and write disjoint cells of grid B, so their blocks run side by side
// (the ALU-heavy interface groups overlap the bandwidth-bound liquid waves).
// Blocks [0, gen) take interface cells, [gen, gen + bord) the liquid cells
// next to walls or obstacles, the rest the liquid chunks.
// (Block b of nb blocks of one run; the kernels below are written this way so
// that one launch can also serve many runs, each with its own block range.)
// After a step that flagged an instability, the run stops: every step kernel
// of the later steps returns at once (halt word of the step's slot, written
// only by the previous step's k_compact, so all blocks of a launch see the same
// value), and the state stays that of the failing step.
__device__ __forceinline__ bool halted(const Dev& d) { return d.cnt[CNT_HALT0 + (d.step & 1)] != 0; }

template <int S, int Q, bool TRT, bool BUF, bool AA>
__device__ __forceinline__ void stream_body(const Dev& d, int b, int nb, int gen, int bord) {
  // the halt word and the list counts in one round trip
  const int32_t halt = d.cnt[CNT_HALT0 + (d.step & 1)];
  const int32_t n_if = d.cnt[CNT_IF], n_gen = d.cnt[CNT_GEN], n_conv = d.cnt[CNT_CONV];
  const int32_t n_ch = d.cnt[CNT_CHUNKS];
  const int32_t err = AA ? d.cnt[CNT_ERR] : 0;
  if (halt != 0) return;
  // in place: the last conversions outgrew a stash buffer; the step does
  // nothing (no marks, empty new-cell lists) and the run halts after it
  const bool stash_full = AA && (n_if > d.stash_cap || (err & ERR_STASH) != 0);
  if (b == 0 && threadIdx.x == 0) {
    d.cnt[CNT_MARK0 + ((d.step + 1) & 1)] = 0;  // mark slot of the next step
    d.cnt[CNT_NG] = 0;                          // new-cell lists of this step
    d.cnt[CNT_NL] = 0;
    if (AA) {
      d.cnt[CNT_SBASE] = n_if;  // stash entries of the next step's buffer
      d.cnt[CNT_SNEW] = 0;
      if (stash_full) atomicOr(&d.cnt[CNT_ERR], ERR_STASH);
    }
  }
  if (stash_full) return;
  if (b < gen)
    generic_role<S, Q, TRT, AA>(d, b, gen, n_if);
  else if (b < gen + bord)
    border_role<S, Q, TRT, AA>(d, b - gen, bord, n_gen, n_conv);
  else
    liquid_role<S, Q, TRT, BUF, AA>(d, b - gen - bord, nb - gen - bord, n_ch);
}

template <int S, int Q, bool TRT, bool BUF, bool AA>
__global__ __launch_bounds__(kBlock) void k_stream(Dev d, int gen, int bord) {
  stream_body<S, Q, TRT, BUF, AA>(d, (int)blockIdx.x, (int)gridDim.x, gen, bord);
}

// In-place layout, at creation (after the interface list is built): each
// interface cell's q own post-collision populations, copied into entry `item`
// (its list position) of the stash buffer of the current step parity, and
// prevpos[c] = item. From then on the streaming launch keeps the buffers.
template <int S, int Q>
__global__ __launch_bounds__(kBlock) void k_stash_init(Dev d) {
  using St = Store<S, Q>;
  const int32_t nif = d.cnt[CNT_IF];
  if (nif > d.stash_cap) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&d.cnt[CNT_ERR], ERR_STASH);
    return;
  }
  const int par = (int)(d.step & 1);
  const typename St::T* F = static_cast<const typename St::T*>(d.fA);
  const int l = threadIdx.x & (kG - 1);
  const int k = l < Q ? l : 0;
  const int64_t groups = (int64_t)gridDim.x * (kBlock / kG);
  for (int64_t it = (int64_t)blockIdx.x * (kBlock / kG) + threadIdx.x / kG; it < nif; it += groups) {
    const int32_t e = d.if_list[it];
    const int64_t c = list_cell(e);
    if (l < Q)
      St::st(stash_buf<S, Q>(d, par), it * Q + k, k,
             St::ld(F, own_slot<Q>(d, c, list_border(e) ? F_BORDER : (uint8_t)0, k, par), k));
    if (l == 0) d.prevpos[c] = (int32_t)it;
  }
}

// In-place layout, at creation: every non-obstacle cell marks the slots of its
// q arrivals in a bitmap (bits over q * stride elements, cleared by the
// caller); a slot marked twice sets ERR_SLOTS (walls and obstacles for which
// pull streaming takes some population twice; such runs need two grids).
template <int Q>
__global__ __launch_bounds__(kBlock) void k_aa_check(Dev d, uint32_t* bits) {
  const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (c >= d.g.N) return;
  if (is_obst(d.flags[c] & T_MASK)) return;
  int x, y, z;
  coords(d.g, c, x, y, z);
  for (int k = 0; k < Q; ++k) {
    const int64_t e = aa_slot<Q>(d.g, d.flags, x, y, z, c, k);
    const uint32_t bit = 1u << (uint32_t)(e & 31);
    if (atomicOr(&bits[e >> 5], bit) & bit) atomicOr(&d.cnt[CNT_ERR], ERR_SLOTS);
  }
}

// ---------------------------------------------------------------------------
// k_retype and k_compact: new types from the marks, then the lists.
// ---------------------------------------------------------------------------
// Conversion of the marked cells (Sec. 2.2), one group of 32 lanes per cell
// of the mark list, lane k looking at the neighbour x + c_k. A to-liquid mark
// turns the cell liquid and its gas neighbours interface. A to-gas mark is
// dropped when some neighbour carries a to-liquid mark (separating liquid from
// gas comes first); otherwise the cell turns gas and its liquid neighbours
// interface. A surviving to-gas cell has no to-liquid neighbour, so no cell is
// asked to become two things; a cell reached from several marked cells gets
// the same byte from each, whatever the order of the groups.
// Turns cell j, if it still has type `from` (gas or liquid), into a new
// interface cell with the transient bit `bit` (static bits kept) by a
// compare-and-swap on the 32-bit word holding its flag byte; true for the one
// caller that made the change. `seen` is the caller's earlier read of that
// word, the first expected value (a stale one only makes the exchange fail
// once and retry with the current word); plain byte stores to the other bytes
// of the word only make the exchange retry.
__device__ __forceinline__ bool set_new_type(uint8_t* flags, int64_t j, uint8_t from, uint8_t bit,
                                             uint32_t seen) {
  uint32_t* w = reinterpret_cast<uint32_t*>(flags + (j & ~(int64_t)3));
  const int sh = 8 * (int)(j & 3);
  uint32_t old = seen;
  for (;;) {
    const uint8_t f = (uint8_t)(old >> sh);
    if ((f & T_MASK) != from) return false;
    const uint8_t nf = (uint8_t)((f & F_STATIC) | T_IF | bit);
    const uint32_t want = (old & ~(0xffu << sh)) | ((uint32_t)nf << sh);
    if (__hip_atomic_compare_exchange_strong(w, &old, want, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT))
      return true;
  }
}

// Appends the cells j of the calling wave's lanes with `take` to a list whose
// length is counter *n: one atomic add per wave (a step with many conversions
// lists thousands of cells, and adds to one address serialise), lanes in
// ascending order after the wave's base. The order of a list's entries is
// not used by any result.
__device__ __forceinline__ void wave_append(int32_t* list, int32_t* n, bool take, int64_t j) {
  const uint64_t won = __ballot(take);
  if (won == 0ull) return;
  const int lane = (int)(threadIdx.x & 63);
  const int leader = __ffsll((long long)won) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(n, __popcll(won));
  base = __shfl(base, leader, 64);
  if (take) list[base + __popcll(won & ((1ull << lane) - 1ull))] = (int32_t)j;
}

// Block 0 also starts the compaction that follows: ticket counter reset and,
// when the compaction will run, a new epoch for its tile-status words.
template <int Q>
__device__ __forceinline__ void retype_body(const Dev& d, int b, int nb, int rebuild_only) {
  if (!rebuild_only && halted(d)) return;
  const int nmk = rebuild_only ? 0 : d.cnt[CNT_MARK0 + (d.step & 1)];
  if (b == 0 && threadIdx.x == 0) {
    d.cnt[CNT_TICKET] = 0;
    if (rebuild_only || nmk > 0) d.cnt[CNT_EPOCH] += 1;
    d.cnt[CNT_SMOOTH] += 1;  // the next step's smoothing-tile tag
  }
  const int l = threadIdx.x & (kG - 1);
  const int ngroups = nb * (kBlock / kG);
  for (int item = b * (kBlock / kG) + threadIdx.x / kG; item < nmk; item += ngroups) {
    const int64_t c = d.mark_list[item];
    const uint8_t mk = d.mark[c];
    int x, y, z;
    coords(d.g, c, x, y, z);
    int64_t j = -1;
    if (l > 0 && l < Q) {
      int w;
      j = nb_index(d.g, x, y, z, cxd(l), cyd(l), czd(l), &w);
    }
    const uint8_t mj = j >= 0 ? d.mark[j] : (uint8_t)MK_NONE;
    // the aligned word holding the neighbour's flag byte (the flag array is
    // padded past its last cell), so that a compare-and-swap below needs no
    // read of its own
    const uint32_t wj = j >= 0 ? *reinterpret_cast<const uint32_t*>(d.flags + (j & ~(int64_t)3)) : 0u;
    const uint8_t fj = (uint8_t)(wj >> (8 * (int)(j & 3)));
    const bool nb_liq_mark = gballot(mj == MK_L) != 0u;
    // (the list appends are made by the whole wave, both groups together)
    bool new_gas = false, new_liq = false;
    if (mk == MK_L) {
      if (l == 0) d.flags[c] = (uint8_t)((d.flags[c] & F_STATIC) | T_LIQ | F_CONV);
      // the one group whose exchange turns the gas byte into an interface
      // byte lists the cell for its reinitialisation
      new_gas = j >= 0 && (fj & T_MASK) == T_GAS && set_new_type(d.flags, j, T_GAS, F_NEW_GAS, wj);
    } else if (mk == MK_G && !nb_liq_mark) {
      if (l == 0) d.flags[c] = (uint8_t)((d.flags[c] & F_STATIC) | T_GAS | F_CONV);
      new_liq = j >= 0 && (fj & T_MASK) == T_LIQ && set_new_type(d.flags, j, T_LIQ, F_NEW_LIQ, wj);
    }
    wave_append(d.ng_list, &d.cnt[CNT_NG], new_gas, j);
    wave_append(d.nl_list, &d.cnt[CNT_NL], new_liq, j);
  }
}

template <int Q>
__global__ __launch_bounds__(kBlock) void k_retype(Dev d, int rebuild_only) {
  retype_body<Q>(d, (int)blockIdx.x, (int)gridDim.x, rebuild_only);
}

// Block-wide exclusive scan of a per-thread count (wave prefix by shuffles,
// wave totals through LDS). Returns the prefix; *total receives the block sum.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* sh, uint32_t* total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(inc, o, 64);
    if (lane >= o) inc += t;
  }
  if (lane == 63) sh[wv] = inc;
  __syncthreads();
  uint32_t before = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    if (w < wv) before += sh[w];
    tot += sh[w];
  }
  __syncthreads();
  *total = tot;
  return before + inc - v;
}

// Inclusive prefix sum within each 16-lane row (DPP row shifts by 1, 2, 4, 8;
// lanes shifted in from outside the row read 0).
__device__ __forceinline__ uint32_t row_scan(uint32_t x) {
  int v = (int)x;
  v += dpp32<0x111>(v);
  v += dpp32<0x112>(v);
  v += dpp32<0x114>(v);
  v += dpp32<0x118>(v);
  return (uint32_t)v;
}

// Sum over the 64 lanes of the wave (integer): the 32-lane group sum, then
// both halves read as scalars.
__device__ __forceinline__ uint32_t wave_sum(uint32_t x) {
  int v = (int)x;
  v += dpp32<kDppXor1>(v);
  v += dpp32<kDppXor2>(v);
  v += dpp32<kDppHalfMirror>(v);
  v += dpp32<kDppMirror>(v);
  v += __builtin_amdgcn_ds_swizzle(v, kSwzXor16);
  return (uint32_t)(__builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 32));
}

// The block scan for four counts at once, packed two to a 32-bit word in
// 16-bit fields (every prefix and the total of each count below 2^16, so no
// sum carries into the next field or word): row scans by DPP, the rows of a
// wave joined by scalar reads of their totals, the waves through LDS.
template <int NT>
__device__ __forceinline__ void block_excl_scan4(const uint32_t v[4], uint32_t (*sh)[NT / 64], uint32_t pre[4],
                                                 uint32_t tot[4]) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint32_t p[2] = {v[0] | (v[1] << 16), v[2] | (v[3] << 16)};
  uint32_t inc[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    uint32_t x = row_scan(p[h]);
    const uint32_t r0 = __builtin_amdgcn_readlane(x, 15), r1 = __builtin_amdgcn_readlane(x, 31),
                   r2 = __builtin_amdgcn_readlane(x, 47);
    const int row = lane >> 4;
    x += (row >= 1 ? r0 : 0u) + (row >= 2 ? r1 : 0u) + (row >= 3 ? r2 : 0u);
    inc[h] = x;
    if (lane == 63) sh[h][wv] = x;
  }
  __syncthreads();
  uint32_t before[2] = {0, 0}, all[2] = {0, 0};
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (w < wv) before[h] += sh[h][w];
      all[h] += sh[h][w];
    }
  }
  __syncthreads();
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const uint32_t ex = before[h] + inc[h] - p[h];
    pre[2 * h] = ex & 0xffffu;
    pre[2 * h + 1] = ex >> 16;
    tot[2 * h] = all[h] & 0xffffu;
    tot[2 * h + 1] = all[h] >> 16;
  }
}

// Per-byte tests on four flag bytes at once (one 32-bit word): a 4-bit mask
// of the bytes whose bits under `mask` equal `val` (an exact zero-byte test:
// no carry crosses a byte), and of the bytes with bit `bit` set.
__device__ __forceinline__ uint32_t bytes_eq4(uint32_t w, uint32_t mask, uint32_t val) {
  const uint32_t x = (w & (mask * 0x01010101u)) ^ (val * 0x01010101u);
  const uint32_t z = ~(((x & 0x7f7f7f7fu) + 0x7f7f7f7fu) | x | 0x7f7f7f7fu);  // 0x80 in the zero bytes
  // the byte-top bits 7, 15, 23, 31 gathered into bits 21..24 by one product
  return (((z >> 7) * 0x00204081u) >> 21) & 0xfu;
}
static_assert(F_CONV == (1u << 6), "bytes_bit4 below tests bit 6");
__device__ __forceinline__ uint32_t bytes_bit4(uint32_t w, int bit) {
  return ((((w >> bit) & 0x01010101u) * 0x00204081u) >> 21) & 0xfu;
}

__device__ __forceinline__ uint32_t mask_of(const uint4& v, int64_t b0, int64_t N, int which) {
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
  uint32_t m = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    uint32_t n;
    if (which == 0) n = bytes_eq4(w[q], T_MASK, T_IF);
    else if (which == 1) n = bytes_bit4(w[q], 6);  // F_CONV
    else if (which == 2) n = bytes_eq4(w[q], T_MASK | F_COMPLEX, T_LIQ);
    else if (which == 3) n = bytes_eq4(w[q], T_MASK | F_COMPLEX, T_LIQ | F_COMPLEX);
    else n = bytes_eq4(w[q], T_MASK | F_BORDER, T_IF | F_BORDER);
    m |= n << (4 * q);
  }
  // the cells of the vector inside the grid
  const uint32_t lim = b0 + 16 <= N ? 0xffffu : (b0 < N ? (1u << (uint32_t)(N - b0)) - 1u : 0u);
  return m & lim;
}

__device__ __forceinline__ uint4 load_flags16(const uint8_t* flags, int64_t b0, int64_t N) {
  if (b0 + 16 <= N) return *reinterpret_cast<const uint4*>(flags + b0);
  union {
    uint4 v;
    uint8_t b[16];
  } u;
  u.v = make_uint4(0, 0, 0, 0);
  for (int j = 0; j < 16; ++j)
    if (b0 + j < N) u.b[j] = flags[b0 + j];
  return u.v;
}

// Flux class of an interface cell from the types around it.
__device__ __forceinline__ uint8_t flux_class(bool has_liq, bool has_gas) {
  return (!has_liq && has_gas) ? CLS_NOLIQ : ((!has_gas && has_liq) ? CLS_NOGAS : CLS_STD);
}

// Interface neighbours (new types) of cell z, its q-1 flag loads issued
// together (a wall neighbour reads z itself and is ignored).
template <int Q>
__device__ __forceinline__ int count_if_nb(const Dev& d, int64_t z, uint8_t fz) {
  if (!(fz & F_BORDER)) {
    // the whole box lies inside the domain and holds no obstacle: plain
    // offsets, no per-direction wall tests between the loads
    const int64_t nx = d.g.nx, nxy = (int64_t)d.g.nx * d.g.ny;
    int n = 0;
#pragma unroll
    for (int k = 1; k < Q; ++k) n += ((d.flags[z + kCX[k] + kCY[k] * nx + kCZ[k] * nxy] & T_MASK) == T_IF) ? 1 : 0;
    return n;
  }
  int x, y, zz;
  coords(d.g, z, x, y, zz);
  uint8_t t[Q];
#pragma unroll
  for (int k = 1; k < Q; ++k) {
    int w;
    const int64_t j = nb_index(d.g, x, y, zz, kCX[k], kCY[k], kCZ[k], &w);
    const uint8_t f = d.flags[j >= 0 ? j : z];
    t[k] = j >= 0 ? (uint8_t)(f & T_MASK) : (uint8_t)T_NOSLIP;
  }
  int n = 0;
#pragma unroll
  for (int k = 1; k < Q; ++k) n += (t[k] == T_IF) ? 1 : 0;
  return n;
}

// Excess mass of a converted cell z (flag byte fz) (Sec. 2.2): m - rho when
// it filled, m when it emptied; each of its interface neighbours (new types)
// receives an equal share.
template <int Q>
__device__ __forceinline__ double excess_share(const Dev& d, int64_t z, uint8_t fz, bool filled) {
  const double mz = d.m[z], rz = d.rho_if[z];
  const int n = count_if_nb<Q>(d, z, fz);
  return (filled ? mz - rz : mz) / (double)n;
}

// A marked cell z, by a group of 32 lanes (lane l looks at z + c_l): if it
// converted, with no interface neighbour (new types) its excess mass is
// booked as lost, its mark is cleared and its fill level set to 1 or 0.
template <int Q>
__device__ __forceinline__ void finish_converted(const Dev& d, int64_t z, int l) {
  const Geom& g = d.g;
  int x, y, zz;
  coords(g, z, x, y, zz);
  const uint8_t fz = d.flags[z];
  bool nb_if = false;
  if (l > 0 && l < Q) {
    int w;
    const int64_t j = nb_index(g, x, y, zz, cxd(l), cyd(l), czd(l), &w);
    const uint8_t f = d.flags[j >= 0 ? j : z];
    nb_if = j >= 0 && (f & T_MASK) == T_IF;
  }
  const double mz = d.m[z], rz = d.rho_if[z];
  const uint32_t nif = gballot(nb_if);
  if (!(fz & F_CONV) || l != 0) return;
  const bool liq = (fz & T_MASK) == T_LIQ;
  if (nif == 0u) d.lost[z] += liq ? mz - rz : mz;
  d.mark[z] = MK_NONE;
  d.phiA[z] = liq ? 1.0 : 0.0;
  d.phiB[z] = liq ? 1.0 : 0.0;
}

// A new interface cell c from gas (Sec. 2.2), by a group of 32 lanes, lane k
// looking at the neighbour x + c_k: the equilibrium of the mean density and
// velocity of its liquid and old interface neighbours (post-collision moments
// of this step), then the collision of this step; rho = the mean density, m =
// the shares of its converted neighbours (added in direction order), fill
// level m / rho, flux classes from the neighbour types.
template <int S, int Q, bool TRT, bool AA>
__device__ __forceinline__ void reinit_from_gas(const Dev& d, int64_t c, int l) {
  using St = Store<S, Q>;
  using T = typename St::T;
  using R = typename St::R;
  constexpr bool SH = St::kShift;
  T* B = static_cast<T*>(d.fB);
  const Geom& g = d.g;
  const int64_t stride = g.stride;
  const bool act = l < Q;
  const int k = act ? l : 0;
  int x, y, z;
  coords(g, c, x, y, z);
  int64_t j = -1;
  uint8_t fj = 0;
  if (act && l > 0) {
    int w;
    j = nb_index(g, x, y, z, cxd(k), cyd(k), czd(k), &w);
    fj = d.flags[j >= 0 ? j : c];
  }
  const int tj = j >= 0 ? (fj & T_MASK) : -1;
  const bool use = j >= 0 && is_fluid(tj) && !(fj & F_NEW_GAS);
  const bool cv = j >= 0 && (fj & F_CONV);
  // (in place: the state after this step's streaming has parity step + 1)
  const int par = (int)((d.step + 1) & 1);
  // the excess share of a converted neighbour, requested before the
  // neighbours' populations, so that both sets of loads are in flight at once
  const double share = cv ? excess_share<Q>(d, j, fj, tj == T_LIQ) : 0.0;
  R r = R(0), a = R(0), b = R(0), cc = R(0);
  // in place after an even step, a neighbour next to walls or obstacles keeps
  // its populations in slots that need aa_slot: the group reads them one
  // neighbour at a time, lane i taking population i, and the lane of that
  // neighbour sums them in post_moments' order (few cells; per lane and
  // unrolled, the slot resolution would hold too many registers)
  const bool slow = AA && use && par && (fj & F_BORDER);
  if constexpr (AA) {
    uint32_t need = gballot(slow);
    while (need) {
      const int m = __ffs(need) - 1;
      need &= need - 1;
      const int64_t jm = (int64_t)__shfl((int)j, m, kG);
      const uint8_t fm = (uint8_t)__shfl((int)fj, m, kG);
      const R v = l < Q ? St::ld(B, own_slot<Q>(d, jm, fm, l, par), l) : R(0);
      R s0 = R(0), s1 = R(0), s2 = R(0), s3 = R(0);
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const R vi = __shfl(v, i, kG);
        s0 += vi;
        if (cxd(i) > 0) s1 += vi;
        if (cxd(i) < 0) s1 += -vi;
        if (cyd(i) > 0) s2 += vi;
        if (cyd(i) < 0) s2 += -vi;
        if (czd(i) > 0) s3 += vi;
        if (czd(i) < 0) s3 += -vi;
      }
      if (l == m) {
        r = SH ? R(1) + s0 : s0;
        a = (s1 - R(0.5) * (r * R(d.gx))) / r;
        b = (s2 - R(0.5) * (r * R(d.gy))) / r;
        cc = (s3 - R(0.5) * (r * R(d.gz))) / r;
      }
    }
  }
  if (use && !slow) {
    R fn[Q];
    if (AA && par) {
      const int64_t nx = g.nx, nxy = (int64_t)g.nx * g.ny;
#pragma unroll
      for (int i = 0; i < Q; ++i)
        fn[i] = St::ld(B, opp(i) * stride + j + cxd(i) + cyd(i) * nx + czd(i) * nxy, i);
    } else {
#pragma unroll
      for (int i = 0; i < Q; ++i) fn[i] = St::ld(B, i * stride + j, i);
    }
    post_moments<R, Q, SH>(fn, R(d.gx), R(d.gy), R(d.gz), r, a, b, cc);
  }
  const uint32_t liq = gballot(tj == T_LIQ), gas = gballot(tj == T_GAS), cvm = gballot(cv);
  const int cnt = __popc(gballot(use));
  const R rb = gsum(r, Q) / R(cnt);
  const R ub0 = gsum(a, Q) / R(cnt), ub1 = gsum(b, Q) / R(cnt), ub2 = gsum(cc, Q) / R(cnt);
  const R usq = ub0 * ub0 + ub1 * ub1 + ub2 * ub2;
  const R fe = feq_k<R, Q, SH>(k, rb, rb - R(1), cdot<R>(cxd(k), cyd(k), czd(k), ub0, ub1, ub2), usq);
  CollideParams<R> cp{R(d.omega), R(d.omega_m), R(d.gx), R(d.gy), R(d.gz), R(d.tau0), R(d.lambda), R(d.cs)};
  R rr, vx, vy, vz;
  const R fs = gcollide<R, Q, TRT, SH>(fe, l, cp, rr, vx, vy, vz);
  if constexpr (AA) {
    if (act) St::st(B, own_slot<Q>(d, c, par ? d.flags[c] : (uint8_t)0, k, par), k, fs);
  } else {
    if (act) St::st(B, k * stride + c, k, fs);
  }
  if constexpr (AA) {
    // (in place: the next step reads the cell's own populations from the stash)
    const int32_t pos = new_stash_entry(d, c, l);
    if (act && pos >= 0) St::st(stash_buf<S, Q>(d, par), (int64_t)pos * Q + k, k, fs);
  }
  double mass = 0.0;
  for (int i = 1; i < Q; ++i) {
    const double si = __shfl(share, i, kG);
    if ((cvm >> i) & 1u) mass += si;
  }
  if (l == 0) {
    const double rho_n = (double)rb;
    d.m[c] = mass;
    d.rho_if[c] = rho_n;
    d.phiB[c] = mass / rho_n;
    d.cls[c] = flux_class(liq != 0u, gas != 0u);
  }
}

// Completion of the cell c = z + c_k (k = 0: z itself) for a source z of this
// step (a cell that carries a transient bit: converted, or new interface),
// by a group of 32 lanes (lane l looks at c + c_l), when c is an old interface
// cell or a new one from liquid: flux classes from the new neighbour types; a
// new cell from liquid takes rho = m = the density of its populations; the
// shares of converted neighbours (each computed by its lane) are added in
// direction order; fill level m / rho. Of all pairs that reach c, the one
// whose source is the first source around c in direction order (c itself
// first) completes it; the others stop after the flag loads. Pairs from the
// mark list whose cell did not convert are no source and never complete.
template <int S, int Q, bool TRT, bool AA>
__device__ __forceinline__ void complete_pair(const Dev& d, int64_t z, int k, int l) {
  using St = Store<S, Q>;
  using T = typename St::T;
  const Geom& g = d.g;
  int x, y, zz;
  coords(g, z, x, y, zz);
  int64_t c = z;
  if (k > 0) {
    int w;
    c = nb_index(g, x, y, zz, cxd(k), cyd(k), czd(k), &w);
    if (c < 0) return;
    coords(g, c, x, y, zz);
  }
  const bool act = l > 0 && l < Q;
  int64_t j = -1;
  if (act) {
    int w;
    j = nb_index(g, x, y, zz, cxd(l), cyd(l), czd(l), &w);
  }
  const uint8_t fc = d.flags[c];
  const uint8_t f = d.flags[j >= 0 ? j : c];
  const double m_old = d.m[c], r_old = d.rho_if[c];
  if ((fc & T_MASK) != T_IF || (fc & F_NEW_GAS)) return;
  const int t = j >= 0 ? (f & T_MASK) : -1;
  const bool cv = j >= 0 && (f & F_CONV);
  const uint32_t liq = gballot(t == T_LIQ), gas = gballot(t == T_GAS), cvm = gballot(cv);
  const uint32_t src = gballot(j >= 0 && (f & F_TRANSIENT)) | ((fc & F_NEW_LIQ) ? 1u : 0u);
  if (__ffs(src) - 1 != opp(k)) return;  // another pair completes c (or z is no source)
  const double share = cv ? excess_share<Q>(d, j, f, t == T_LIQ) : 0.0;
  const bool new_liq = (fc & F_NEW_LIQ) != 0;
  const int par = (int)((d.step + 1) & 1);
  double pop = 0.0;
  typename St::R popr = typename St::R(0);
  if (new_liq && l < Q) {
    popr = St::ld(static_cast<const T*>(d.fB), AA ? own_slot<Q>(d, c, fc, l, par) : l * g.stride + c, l);
    pop = (double)popr;
  }
  if (AA && new_liq) {
    // (in place: the next step reads the cell's own populations from the stash)
    const int32_t pos = new_stash_entry(d, c, l);
    if (l < Q && pos >= 0) St::st(stash_buf<S, Q>(d, par), (int64_t)pos * Q + l, l, popr);
  }
  double mass = m_old, rho_n = r_old;
  if (new_liq) {
    double r = 0.0;
    for (int i = 0; i < Q; ++i) r += __shfl(pop, i, kG);
    rho_n = (St::kShift ? 1.0 : 0.0) + r;
    mass = rho_n;
  }
  for (int i = 1; i < Q; ++i) {
    const double si = __shfl(share, i, kG);
    if ((cvm >> i) & 1u) mass += si;
  }
  if (l != 0) return;
  d.cls[c] = flux_class(liq != 0u, gas != 0u);
  if (!new_liq && cvm == 0u) return;  // mass and fill level unchanged
  d.m[c] = mass;
  d.rho_if[c] = rho_n;
  d.phiB[c] = mass / rho_n;
}

// Tile status: two 64-bit words per tile, [epoch:16 | count:24 | count:24],
// written once per compaction by the tile and read by every later tile.
__device__ __forceinline__ unsigned long long pack2(uint32_t epoch, uint32_t a, uint32_t b) {
  return ((unsigned long long)(epoch & 0xffffu) << 48) | ((unsigned long long)(a & 0xffffffu) << 24) |
         (unsigned long long)(b & 0xffffffu);
}

// List compaction. A tile is 1024 threads times `per` cells (per = 16 times a
// power of two, chosen by the host so that there are at most kMaxTiles
// tiles); thread t owns the cells [per t, per t + per) of the tile, read as
// 16-byte vectors. The interface list, the converted list, the chunk list
// (64-cell chunks with liquid cells away from walls) and the list of COMPLEX
// liquid cells are compacted in ascending cell order in one pass: each tile
// publishes its four counts at once, then sums the published counts of all
// earlier tiles (whole block, one load round; a tile's ticket is taken in
// launch order, so its predecessors are already running) and writes its
// entries at the resulting offsets. The status words carry the compaction's
// epoch, so they never need clearing; their only payload is the counts
// themselves, so relaxed device-scope atomics suffice. The wait for a
// predecessor is bounded: on expiry the scan error bit is set and the kernel
// completes (with a wrong list, reported by the host). Skipped in a step
// without marks (the lists are unchanged then).
// The first `workers` blocks complete the conversion beside the compaction:
// converted cells, new interface cells, and the interface cells next to any
// of them. Each of these reads only flags, and masses and populations of
// cells other than the ones written in this launch.
template <int S, int Q, bool TRT, bool AA>
__device__ __forceinline__ void compact_body(const Dev& d, int b, int nb, int rebuild_only, int per,
                                             int workers) {
  __shared__ int s_tile, s_run;
  __shared__ uint32_t s_epoch;
  __shared__ uint32_t s_scan[4][kCompBlock / 64];
  __shared__ uint32_t s_scan4[2][kCompBlock / 64];
  __shared__ uint32_t s_red[4][kCompBlock / 64];
  // the next step's halt word: this step's, or set by an instability flagged
  // in this step (its slot is not read by this launch)
  if (!rebuild_only && b == 0 && threadIdx.x == 0)
    d.cnt[CNT_HALT0 + ((d.step + 1) & 1)] =
        (d.cnt[CNT_HALT0 + (d.step & 1)] != 0 || (d.cnt[CNT_ERR] & (ERR_UNSTABLE | ERR_STASH)) != 0) ? 1 : 0;
  if (!rebuild_only && halted(d)) return;
  if (b < workers) {
    // worker blocks, beside the compaction, over one index space of 32-lane
    // groups (at typical conversion rates about one item per group, so that
    // all items proceed at once): the new interface cells from gas
    // (reinitialisation), the marked cells (finished if they converted), and
    // the (source, direction) pairs of the completion, sources being the
    // converted and the new cells
    if (rebuild_only) return;
    const int nmk = d.cnt[CNT_MARK0 + (d.step & 1)];
    const int nng = d.cnt[CNT_NG];
    const int nnl = d.cnt[CNT_NL];
    // (every item is a 32-lane group; the start and the stride are multiples
    // of 32, so every condition below is uniform over a group)
    const int64_t g_cv = (int64_t)nng + nmk;
    const int64_t g_all = g_cv + ((int64_t)nmk + nng + nnl) * Q;
    const int64_t stride = (int64_t)workers * kCompBlock;
    const int l = threadIdx.x & (kG - 1);
    // (two loops over the thread's indices of the one space: the first ends
    // where the second begins, so a thread with one item does only one of them)
    int64_t it = (int64_t)b * kCompBlock + threadIdx.x;
    for (; it < g_cv * kG; it += stride) {
      const int64_t gi = it / kG;
      if (gi < nng)
        reinit_from_gas<S, Q, TRT, AA>(d, d.ng_list[gi], l);
      else
        finish_converted<Q>(d, d.mark_list[gi - nng], l);
    }
    for (; it < g_all * kG; it += stride) {
      const int64_t pr = it / kG - g_cv;
      const int64_t si = pr / Q;
      const int k = (int)(pr - si * Q);
      int64_t z;
      if (si < nmk)
        z = d.mark_list[si];
      else if (si < (int64_t)nmk + nng)
        z = d.ng_list[si - nmk];
      else
        z = d.nl_list[si - nmk - nng];
      complete_pair<S, Q, TRT, AA>(d, z, k, l);
    }
    return;
  }
  // the first 16 flag bytes of this thread, for the tile that the launch
  // order gives the block, requested before the ticket round trip (the ticket
  // almost always agrees; when it does not, they are loaded again)
  constexpr int kBatch = 4;
  const int64_t N = d.g.N;
  const int nvec = per / 16;
  const int spec = b - workers;
  uint4 first;
  {
    const int64_t b0 = ((int64_t)spec * kCompBlock + threadIdx.x) * per;
    first = b0 < N ? load_flags16(d.flags, b0, N) : make_uint4(0, 0, 0, 0);
  }
  if (threadIdx.x == 0) {
    // the mark count, the epoch and the ticket in one round trip (a ticket
    // taken in a step without marks is harmless: the counter is reset before
    // every compaction launch)
    const int run = rebuild_only ? 1 : d.cnt[CNT_MARK0 + (d.step & 1)];
    const uint32_t ep = (uint32_t)d.cnt[CNT_EPOCH];
    s_tile = atomicAdd(&d.cnt[CNT_TICKET], 1);
    s_run = run;
    s_epoch = ep;
  }
  __syncthreads();
  if (s_run == 0) return;
  const int tile = s_tile;
  const uint32_t epoch = s_epoch;
  const int64_t base = ((int64_t)tile * kCompBlock + threadIdx.x) * per;
  if (tile != spec) first = base < N ? load_flags16(d.flags, base, N) : make_uint4(0, 0, 0, 0);
  // threads per 64-cell chunk (per < 64), else chunks per thread
  const int tpc = per < 64 ? 64 / per : 1;
  // pass 1: masks and counts, in batches of kBatch 16-byte vectors requested
  // together; the masks of the first batch are kept for pass 2
  uint32_t keep[5][kBatch];  // the four lists, and interface cells with the BORDER bit
  uint32_t c[4] = {0, 0, 0, 0};
  uint32_t own_any = 0;
  uint32_t own_bits = 0;  // (per < 64) liquid-lane mask of this thread's cells
  {
    uint32_t chunk_any = 0;
#pragma unroll 1
    for (int v0 = 0; v0 < nvec; v0 += kBatch) {
      uint4 vec[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int64_t b0 = base + 16 * (v0 + u);
        if (v0 + u == 0)
          vec[u] = first;
        else
          vec[u] = (v0 + u < nvec && b0 < N) ? load_flags16(d.flags, b0, N) : make_uint4(0, 0, 0, 0);
      }
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int64_t b0 = base + 16 * (v0 + u);
        uint32_t m[5] = {0, 0, 0, 0, 0};
        if (v0 + u < nvec && b0 < N) {
#pragma unroll
          for (int i = 0; i < 5; ++i) m[i] = mask_of(vec[u], b0, N, i);
        }
        if (v0 == 0) {
#pragma unroll
          for (int i = 0; i < 5; ++i) keep[i][u] = m[i];
        }
        c[0] += __popc(m[0]);
        c[1] += __popc(m[1]);
        c[3] += __popc(m[3]);
        own_any |= m[2];
        if (per < 64 && v0 + u < nvec) own_bits |= m[2] << (16 * (v0 + u));  // nvec <= 2 here
        chunk_any |= m[2];
        if (per >= 64 && (u & 3) == 3) {
          c[2] += chunk_any ? 1u : 0u;
          chunk_any = 0;
        }
      }
    }
  }
  // chunk count: a chunk shared by tpc threads is counted by the first,
  // which also gathers the chunk's liquid-lane mask
  uint32_t lead_any = own_any ? 1u : 0u;
  uint64_t lead_bits = 0;
  if (per < 64) {
    if (tpc >= 2) lead_any |= __shfl_xor(lead_any, 1, 64);
    if (tpc >= 4) lead_any |= __shfl_xor(lead_any, 2, 64);
    c[2] = ((threadIdx.x % tpc) == 0) ? lead_any : 0u;
    const int lane = threadIdx.x & 63;
    for (int k = 0; k < tpc; ++k) {
      const uint32_t bk = (uint32_t)__shfl((int)own_bits, (lane + k) & 63, 64);
      lead_bits |= (uint64_t)bk << (per * k);
    }
  }
  uint32_t pre[4], tot[4];
  if (per <= 32) {
    // every count of the tile stays below 1024 * 32 < 2^16
    block_excl_scan4<kCompBlock>(c, s_scan4, pre, tot);
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i) pre[i] = block_excl_scan<kCompBlock>(c[i], s_scan[i], &tot[i]);
  }
  unsigned long long* st = d.scan_status;
  if (threadIdx.x == 0) {
    __hip_atomic_store(&st[2 * tile], pack2(epoch, tot[0], tot[1]), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&st[2 * tile + 1], pack2(epoch, tot[2], tot[3]), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
  // sum of the counts of all earlier tiles
  uint32_t acc[4] = {0, 0, 0, 0};
  for (int t = threadIdx.x; t < tile; t += kCompBlock) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      unsigned long long v;
      int spins = 0;
      for (;;) {
        v = __hip_atomic_load(&st[2 * t + h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((uint32_t)(v >> 48) == (epoch & 0xffffu)) break;
        if (++spins > (1 << 22)) {
          atomicOr(&d.cnt[CNT_ERR], ERR_SCAN);
          v = 0;
          break;
        }
        if (spins > 64) __builtin_amdgcn_s_sleep(1);
      }
      acc[2 * h] += (uint32_t)(v >> 24) & 0xffffffu;
      acc[2 * h + 1] += (uint32_t)v & 0xffffffu;
    }
  }
  {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t x = wave_sum(acc[i]);
      if (lane == 0) s_red[i][wv] = x;
    }
  }
  __syncthreads();
  uint32_t off[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    uint32_t e = 0;
#pragma unroll
    for (int w = 0; w < kCompBlock / 64; ++w) e += s_red[i][w];
    off[i] = e + pre[i];
  }
  const uint32_t chunks_end = off[2] + c[2];
  // pass 2: the entries, in ascending order (masks of the first batch kept,
  // later batches reloaded: the flags are still in cache)
  {
    uint32_t chunk_any = 0;
    uint64_t chunk_bits = 0;
#pragma unroll 1
    for (int v0 = 0; v0 < nvec; v0 += kBatch) {
      uint32_t m[5][kBatch];
      if (v0 == 0) {
#pragma unroll
        for (int u = 0; u < kBatch; ++u)
#pragma unroll
          for (int i = 0; i < 5; ++i) m[i][u] = keep[i][u];
      } else {
        uint4 vec[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
          const int64_t b0 = base + 16 * (v0 + u);
          vec[u] = (v0 + u < nvec && b0 < N) ? load_flags16(d.flags, b0, N) : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
          const int64_t b0 = base + 16 * (v0 + u);
          const bool in = v0 + u < nvec && b0 < N;
#pragma unroll
          for (int i = 0; i < 5; ++i) m[i][u] = in ? mask_of(vec[u], b0, N, i) : 0u;
        }
      }
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int64_t b0 = base + 16 * (v0 + u);
        if (v0 + u >= nvec || b0 >= N) break;
        for (uint32_t mm = m[0][u]; mm; mm &= mm - 1) {
          const int j = __builtin_ctz(mm);
          d.if_list[off[0]++] = list_entry(b0 + j, ((m[4][u] >> j) & 1u) != 0);
        }
        for (uint32_t mm = m[1][u]; mm; mm &= mm - 1) d.conv_list[off[1]++] = (int32_t)(b0 + __builtin_ctz(mm));
        for (uint32_t mm = m[3][u]; mm; mm &= mm - 1) d.gen_list[off[3]++] = (int32_t)(b0 + __builtin_ctz(mm));
        if (per >= 64) {
          chunk_any |= m[2][u];
          chunk_bits |= (uint64_t)m[2][u] << (16 * (u & 3));
          if ((u & 3) == 3 || b0 + 16 >= N) {
            if (chunk_any) {
              d.chunk_mask[off[2]] = chunk_bits;
              d.chunk_list[off[2]++] = (int32_t)(b0 / 64);
            }
            chunk_any = 0;
            chunk_bits = 0;
          }
        }
      }
    }
  }
  if (per < 64 && c[2]) {
    d.chunk_mask[off[2]] = lead_bits;
    d.chunk_list[off[2]] = (int32_t)(base / 64);
  }
  if (tile == nb - workers - 1 && threadIdx.x == kCompBlock - 1) {
    d.cnt[CNT_IF] = (int32_t)off[0];
    d.cnt[CNT_CONV] = (int32_t)off[1];
    d.cnt[CNT_GEN] = (int32_t)off[3];
    d.cnt[CNT_CHUNKS] = (int32_t)chunks_end;
  }
}

template <int S, int Q, bool TRT, bool AA>
__global__ __launch_bounds__(kCompBlock) void k_compact(Dev d, int rebuild_only, int per, int workers) {
  compact_body<S, Q, TRT, AA>(d, (int)blockIdx.x, (int)gridDim.x, rebuild_only, per, workers);
}

// The two-grid compaction with two argument words (workers < 0: the rebuild
// at creation, which has no workers): with the record they stay within 512
// bytes, beyond which a launch costs more (the dam-break step is 1 % faster
// than with k_compact's three words). The in-place compaction keeps three:
// with two, its register allocation spilled more and it ran slower.
template <int S, int Q, bool TRT>
__global__ __launch_bounds__(kCompBlock) void k_compact2(Dev d, int per, int workers) {
  compact_body<S, Q, TRT, false>(d, (int)blockIdx.x, (int)gridDim.x, workers < 0 ? 1 : 0, per,
                                 workers < 0 ? 0 : workers);
}

// ---------------------------------------------------------------------------
// k_classes: flux classes of every cell of the interface list from the types
// around it (when a domain is set up; in a step, the compaction's worker
// blocks update the cells whose neighbourhood changed).
// ---------------------------------------------------------------------------
template <int Q>
__global__ __launch_bounds__(kBlock) void k_classes(Dev d) {
  const Geom& g = d.g;
  const int nif = d.cnt[CNT_IF];
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < nif; i += gridDim.x * kBlock) {
    const int64_t c = list_cell(d.if_list[i]);
    int x, y, z;
    coords(g, c, x, y, z);
    bool has_liq = false, has_gas = false;
#pragma unroll
    for (int k = 1; k < Q; ++k) {
      int w;
      const int64_t j = nb_index(g, x, y, z, kCX[k], kCY[k], kCZ[k], &w);
      const int t = j >= 0 ? (d.flags[j] & T_MASK) : (int)T_NOSLIP;
      has_liq |= t == T_LIQ;
      has_gas |= t == T_GAS;
    }
    d.cls[c] = flux_class(has_liq, has_gas);
  }
}

// ---------------------------------------------------------------------------
// Surface tension (Sec. 2.2): K8-smoothed fill level, curvature, gas density.
// ---------------------------------------------------------------------------
// Smoothing tiles: 64 x 4 cells of one plane.
constexpr int kSmoothTX = 64, kSmoothTY = 4;
__host__ __device__ inline int64_t smooth_tiles(int nx, int ny, int nz) {
  return (int64_t)((nx + kSmoothTX - 1) / kSmoothTX) * ((ny + kSmoothTY - 1) / kSmoothTY) * nz;
}

#ifdef FSLBM_HOST_KERNELS
// The curvature reads the smoothed fill level only within two cells of an
// interface cell (the boxes of the normals of its face neighbours). Before
// the smoothing, each interface cell tags the smoothing tiles holding such
// cells (periodic faces wrap, cells beyond a wall are left out); the
// smoothing skips untagged tiles, whose values are never read. The tag is a
// device counter that k_retype advances once per step, after the smoothing,
// so that it changes from step to step under replayed graphs too.
__device__ __forceinline__ int32_t smooth_tag(const Dev& d) { return d.cnt[CNT_SMOOTH] + 1; }

__device__ __forceinline__ void smooth_mark_body(const Dev& d, int b, int nb) {
  const Geom& g = d.g;
  const int nif = d.cnt[CNT_IF];
  const int tiles_x = (g.nx + kSmoothTX - 1) / kSmoothTX, tiles_y = (g.ny + kSmoothTY - 1) / kSmoothTY;
  const int32_t tag = smooth_tag(d);
  const int n[3] = {g.nx, g.ny, g.nz};
  const int tw[3] = {kSmoothTX, kSmoothTY, 1};
  for (int k = b * kBlock + threadIdx.x; k < nif; k += nb * kBlock) {
    const int64_t c = list_cell(d.if_list[k]);
    int p[3];
    coords(g, c, p[0], p[1], p[2]);
    // the tiles covering [p - 2, p + 2] along each axis (at most five)
    int t[3][5], nt[3];
    for (int a = 0; a < 3; ++a) {
      nt[a] = 0;
      for (int o = -2; o <= 2; ++o) {
        int v = p[a] + o;
        if (v < 0 || v >= n[a]) {
          if (face_kind(g, v < 0 ? 2 * a : 2 * a + 1) != BND_PERIODIC) continue;
          v = ((v % n[a]) + n[a]) % n[a];
        }
        const int ti = v / tw[a];
        bool seen = false;
        for (int q = 0; q < nt[a]; ++q) seen |= t[a][q] == ti;
        if (!seen) t[a][nt[a]++] = ti;
      }
    }
    for (int iz = 0; iz < nt[2]; ++iz)
      for (int iy = 0; iy < nt[1]; ++iy)
        for (int ix = 0; ix < nt[0]; ++ix)
          d.smap[((int64_t)t[2][iz] * tiles_y + t[1][iy]) * tiles_x + t[0][ix]] = tag;
  }
}

__global__ __launch_bounds__(kBlock) void k_smooth_mark(Dev d) {
  smooth_mark_body(d, (int)blockIdx.x, (int)gridDim.x);
}

// Smoothed fill level, K(r) = (1 - r^2/4)^4 over the 3x3x3 box (support
// radius 2), obstacles left out and the weights renormalised, of the cells of
// the tagged tiles (every tile when `all`). The block stages a
// (64+2) x (4+2) x (1+2) halo of phi and flags in LDS.
__device__ __forceinline__ void smooth_body(const Dev& d, int bt, bool all) {
  constexpr int TX = kSmoothTX, TY = kSmoothTY;
  __shared__ double s_phi[3][TY + 2][TX + 2];
  __shared__ uint8_t s_obs[3][TY + 2][TX + 2];
  if (!all && d.smap[bt] != smooth_tag(d)) return;
  const Geom& g = d.g;
  const int tiles_x = (g.nx + TX - 1) / TX, tiles_y = (g.ny + TY - 1) / TY;
  const int tz = bt / (tiles_x * tiles_y);
  const int r = bt - tz * tiles_x * tiles_y;
  const int ty0 = (r / tiles_x) * TY, tx0 = (r % tiles_x) * TX;
  for (int e = threadIdx.x; e < 3 * (TY + 2) * (TX + 2); e += kBlock) {
    const int lz = e / ((TY + 2) * (TX + 2));
    const int rr = e - lz * (TY + 2) * (TX + 2);
    const int ly = rr / (TX + 2), lx = rr - ly * (TX + 2);
    int w;
    const int64_t j = wrap_index(g, tx0 + lx - 1, ty0 + ly - 1, tz + lz - 1, &w);
    const bool ob = (j < 0) || is_obst(d.flags[j] & T_MASK);
    s_obs[lz][ly][lx] = ob;
    s_phi[lz][ly][lx] = ob ? 0.0 : d.phiA[j];
  }
  __syncthreads();
  const int lx = threadIdx.x % TX, ly = threadIdx.x / TX;
  const int x = tx0 + lx, y = ty0 + ly;
  if (x >= g.nx || y >= g.ny) return;
  const int64_t c = x + (int64_t)g.nx * (y + (int64_t)g.ny * tz);
  if (is_obst(d.flags[c] & T_MASK)) {
    d.phis[c] = 0.0;
    return;
  }
  double num = 0.0, den = 0.0;
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        if (s_obs[1 + dz][1 + ly + dy][1 + lx + dx]) continue;
        const double r2 = (double)(dx * dx + dy * dy + dz * dz);
        const double b = 1.0 - r2 / 4.0;
        const double k = b * b * b * b;
        num += k * s_phi[1 + dz][1 + ly + dy][1 + lx + dx];
        den += k;
      }
  d.phis[c] = num / den;
}

__global__ __launch_bounds__(kBlock) void k_smooth(Dev d) { smooth_body(d, (int)blockIdx.x, false); }

// kappa = -div(n_hat) by central differences of the unit normals of the face
// neighbours; rho^G = 3 (p^V + sigma kappa).
// One interface cell per 32-lane group. The seven normals (the cell's and its
// six face neighbours') are Parker-Youngs normals (Sec. 2.2) of the smoothed
// fill level: component a at point P is the sum, over the offsets b, c in
// {-1, 0, 1} of the other two axes (in that order), of w_b w_c times the
// difference of the values at P + e_a and P - e_a shifted by (b, c), with
// w = (1, 2, 1) and obstacle or wall points taking P's value; the unit normal
// divides by the Euclidean length. They read 81 points around the cell
// (offsets up to 2 along at most one axis), which the group stages in LDS
// with one load round; lane 3p + a forms component a of normal p.
constexpr int kCurvPts = 125;  // 5x5x5 staging box; 81 of its points are used
__device__ __forceinline__ int curv_slot(int ox, int oy, int oz) { return (ox + 2) + 5 * ((oy + 2) + 5 * (oz + 2)); }

__device__ __forceinline__ void curvature_body(const Dev& d, int b, int nb) {
  __shared__ double s_phi[kBlock / kG][kCurvPts];
  __shared__ uint8_t s_obs[kBlock / kG][kCurvPts];
  const Geom& g = d.g;
  const int nif = d.cnt[CNT_IF];
  const int l = threadIdx.x & (kG - 1);
  const int grp = threadIdx.x / kG;
  double* ph = s_phi[grp];
  uint8_t* ob = s_obs[grp];
  // this lane's normal p (0: the cell, 2a + 1 / 2a + 2: the +a / -a face
  // neighbour) and component
  const int p = l < 21 ? l / 3 : 0, a = l < 21 ? l % 3 : 0;
  const int ea = p == 0 ? 0 : (p - 1) / 2, sg = p == 0 ? 0 : ((p & 1) ? 1 : -1);
  const int px = ea == 0 ? sg : 0, py = ea == 1 ? sg : 0, pz = ea == 2 ? sg : 0;
  const int a1 = (a + 1) % 3, a2 = (a + 2) % 3;
  for (int item = b * (kBlock / kG) + grp; item < nif; item += nb * (kBlock / kG)) {
    const int64_t c = list_cell(d.if_list[item]);
    int x, y, z;
    coords(g, c, x, y, z);
    // stage the points: wall ghosts and obstacle cells are marked (their
    // value is never read); every load of the round is issued at once
#pragma unroll
    for (int sl = l; sl < kCurvPts; sl += kG) {
      const int ox = sl % 5 - 2, oy = (sl / 5) % 5 - 2, oz = sl / 25 - 2;
      const int far = (ox == 2 || ox == -2) + (oy == 2 || oy == -2) + (oz == 2 || oz == -2);
      if (far > 1) continue;
      int w;
      const int64_t j = wrap_index(g, x + ox, y + oy, z + oz, &w);
      const bool o = j < 0 || is_obst(d.flags[j] & T_MASK);
      ob[sl] = o;
      ph[sl] = j < 0 ? 0.0 : d.phis[j];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // component a of the Parker-Youngs normal at the point P of normal p
    const double W[3] = {1.0, 2.0, 1.0};
    const double v0 = ph[curv_slot(px, py, pz)];
    double s = 0.0;
    for (int bb = -1; bb <= 1; ++bb) {
      for (int cc = -1; cc <= 1; ++cc) {
        int dp[3], dm[3];
        dp[a] = 1;
        dm[a] = -1;
        dp[a1] = dm[a1] = bb;
        dp[a2] = dm[a2] = cc;
        const int sp = curv_slot(px + dp[0], py + dp[1], pz + dp[2]);
        const int sm = curv_slot(px + dm[0], py + dm[1], pz + dm[2]);
        const double vp = ob[sp] ? v0 : ph[sp];
        const double vm = ob[sm] ? v0 : ph[sm];
        s += W[bb + 1] * W[cc + 1] * (vp - vm);
      }
    }
    // the unit normal (every lane of normal p forms the same length)
    const int l0 = 3 * p;
    const double n0 = __shfl(s, l0, kG), n1 = __shfl(s, l0 + 1, kG), n2 = __shfl(s, l0 + 2, kG);
    const double len = sqrt(n0 * n0 + n1 * n1 + n2 * n2);
    const double nh = len > 0.0 ? s / len : 0.0;
    // divergence: the face neighbour's normal where it is a fluid cell,
    // else the cell's own
    double div = 0.0;
    for (int e = 0; e < 3; ++e) {
      const double nc = __shfl(nh, e, kG);
      const double np_ = __shfl(nh, 3 * (2 * e + 1) + e, kG);
      const double nm_ = __shfl(nh, 3 * (2 * e + 2) + e, kG);
      const int op = curv_slot(e == 0 ? 1 : 0, e == 1 ? 1 : 0, e == 2 ? 1 : 0);
      const int om = curv_slot(e == 0 ? -1 : 0, e == 1 ? -1 : 0, e == 2 ? -1 : 0);
      div += 0.5 * ((ob[op] ? nc : np_) - (ob[om] ? nc : nm_));
    }
    if (l == 0) {
      const double kappa = -div;
      const double pv = d.bubble == 2 ? d.bpr[d.blab[c]] : d.pV[0];
      d.rhoG[c] = 3.0 * (pv + d.sigma * kappa);
    }
    // (the next item's staging overwrites the points only after every lane
    // has read them)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

__global__ __launch_bounds__(kBlock) void k_curvature(Dev d) {
  curvature_body(d, (int)blockIdx.x, (int)gridDim.x);
}

#endif  // FSLBM_HOST_KERNELS

// ---------------------------------------------------------------------------
// Deterministic FP64 reductions: per-block partials in a fixed tree order, then
// one block sums the partials in order.
// ---------------------------------------------------------------------------
template <int NV>
__device__ __forceinline__ void block_reduce_store(double (&v)[NV], double* out) {
  __shared__ double sh[NV][kBlock];
#pragma unroll
  for (int i = 0; i < NV; ++i) sh[i][threadIdx.x] = v[i];
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
#pragma unroll
      for (int i = 0; i < NV; ++i) sh[i][threadIdx.x] += sh[i][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) out[i] = sh[i][0];
  }
}

// Values per cell: [0] liquid rho, [1] interface m, [2] lost, [3] bubble volume
// contribution, [4] n_liquid, [5] n_interface, [6] n_gas.
constexpr int kRedN = 7;
constexpr int kRedCells = 8192;  // cells per block of the mass reduction
// cells per block of the bubble-volume reduction: four times the mass
// reduction's block count, which the partial buffer (kRedN values per mass
// block) holds
constexpr int kVolCells = kRedCells / 4;
static_assert(kRedN >= 4, "volume partials must fit the partial buffer");
__host__ __device__ inline int64_t red_blocks_of(int64_t N) { return (N + kRedCells - 1) / kRedCells; }
__host__ __device__ inline int64_t vol_blocks_of(int64_t N) { return (N + kVolCells - 1) / kVolCells; }

template <int S, int Q>
__global__ __launch_bounds__(kBlock) void k_reduce_mass(Dev d, int cells_per_block) {
  using St = Store<S, Q>;
  using T = typename St::T;
  const T* A = static_cast<const T*>(d.fA);
  double v[kRedN] = {0, 0, 0, 0, 0, 0, 0};
  const int64_t begin = (int64_t)blockIdx.x * cells_per_block;
  int64_t end = begin + cells_per_block;
  if (end > d.g.N) end = d.g.N;
  for (int64_t c = begin + threadIdx.x; c < end; c += kBlock) {
    const uint8_t fl = d.flags[c];
    const int t = fl & T_MASK;
    if (t == T_LIQ) {
      typename St::R f[Q];
      if (d.aa && (d.step & 1)) {
#pragma unroll
        for (int k = 0; k < Q; ++k) f[k] = St::ld(A, own_slot<Q>(d, c, fl, k, 1), k);
      } else {
#pragma unroll
        for (int k = 0; k < Q; ++k) f[k] = St::ld(A, k * d.g.stride + c, k);
      }
      v[0] += density64<typename St::R, Q, St::kShift>(f);
      v[4] += 1.0;
    } else if (t == T_IF) {
      v[1] += d.m[c];
      v[3] += 1.0 - d.phiA[c];
      v[5] += 1.0;
    } else if (t == T_GAS) {
      v[3] += 1.0;
      v[6] += 1.0;
    }
    v[2] += d.lost[c];
  }
  block_reduce_store<kRedN>(v, d.partial + (int64_t)blockIdx.x * kRedN);
}

#ifdef FSLBM_HOST_KERNELS
// Bubble volume only (sum of 1 - phi over gas and interface cells) from the
// fill levels at t+1; one block then updates p^V = p^V(0) V(0) / V.
__device__ __forceinline__ void reduce_volume_body(const Dev& d, int blk, int cells_per_block) {
  double v[1] = {0.0};
  const int64_t begin = (int64_t)blk * cells_per_block;
  int64_t end = begin + cells_per_block;
  if (end > d.g.N) end = d.g.N;
  for (int64_t c = begin + threadIdx.x; c < end; c += kBlock) {
    const int t = d.flags[c] & T_MASK;
    if (t == T_GAS)
      v[0] += 1.0;
    else if (t == T_IF)
      v[0] += 1.0 - d.phiB[c];
  }
  block_reduce_store<1>(v, d.partial + blk);
}

__global__ __launch_bounds__(kBlock) void k_reduce_volume(Dev d, int cells_per_block) {
  reduce_volume_body(d, (int)blockIdx.x, cells_per_block);
}

// Sum of per-block partials (nv values each) in a fixed order, by one block
// of kBlock threads: thread t adds the partials t, t + kBlock, t + 2 kBlock,
// ... in that order, then the threads' sums are added pairwise in a fixed
// tree. The order depends only on nblocks, so every call on the same
// partials gives the same bits.
constexpr int kSumMaxV = 8;
__device__ __forceinline__ void sum_partials_body(const double* partial, int nblocks, int nv, double* out) {
  __shared__ double sh[kSumMaxV][kBlock];
  double v[kSumMaxV];
#pragma unroll
  for (int i = 0; i < kSumMaxV; ++i) v[i] = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kBlock) {
#pragma unroll
    for (int i = 0; i < kSumMaxV; ++i)
      if (i < nv) v[i] += partial[(int64_t)b * nv + i];
  }
#pragma unroll
  for (int i = 0; i < kSumMaxV; ++i) sh[i][threadIdx.x] = v[i];
  __syncthreads();
  for (int h = kBlock / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
#pragma unroll
      for (int i = 0; i < kSumMaxV; ++i) sh[i][threadIdx.x] += sh[i][threadIdx.x + h];
    }
    __syncthreads();
  }
  if ((int)threadIdx.x < nv) out[threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(kBlock) void k_sum_partials(const double* partial, int nblocks,
                                                         int nv, double* out) {
  sum_partials_body(partial, nblocks, nv, out);
}

// The bubble volume V from the partials of k_reduce_volume, then the
// volume pressure p^V = p^V(0) V(0) / V (Sec. 2.2), or, when the reference
// is set, V(0) = V. pV: [0] p^V, [1] p^V(0), [2] V(0); out receives V.
__device__ __forceinline__ void sum_volume_body(const double* partial, int nblocks, double* out, double* pV,
                                                int set_reference) {
  sum_partials_body(partial, nblocks, 1, out);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (set_reference)
      pV[2] = out[0];
    else
      pV[0] = pV[1] * pV[2] / out[0];
  }
}

__global__ __launch_bounds__(kBlock) void k_sum_volume(const double* partial, int nblocks, double* out,
                                                       double* pV, int set_reference) {
  sum_volume_body(partial, nblocks, out, pV, set_reference);
}

// Report of fslbm_mass_noalloc: r[1..7] hold the sums of the mass reduction;
// r[0] = liquid + interface + lost mass, added as the host does it.
__global__ void k_total_of_report(double* r) {
  if (threadIdx.x == 0) r[0] = r[1] + r[2] + r[3];
}


// ---------------------------------------------------------------------------
// Tracked bubbles (bubble model 2; Sec. 2.2 volume pressure followed through
// coalescence and segmentation). A bubble is a connected set of gas and
// interface cells (lattice neighbours, periodic faces wrap); V = sum of
// 1 - phi; its amount n = p^V V is kept by Boyle's law. After each step the
// bubbles are found again (union-find, each bubble's root its smallest cell
// index); an old bubble hands its amount to the new bubbles holding its
// former cells in proportion to their gas volume, cells new to any bubble
// add volume only, and a bubble without any handed amount starts at p^V(0).
// Of each old bubble, the new bubble with the smallest label among its former
// cells receives the rest of its amount, n_b (1 - R_b / W_b) (R_b: volume of
// its former cells elsewhere), so a bubble that neither merges nor splits
// keeps its amount exactly; the others the shares n_b w / W_b of their cells.
// Seven passes over the grid; sums by atomic adds, combined per wave first.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool bubble_cell(uint8_t f) {
  const int t = f & T_MASK;
  return t == T_GAS || t == T_IF;
}

// A parent always has a smaller index than its child (a root is linked under
// a smaller root by compare-and-swap, and halving replaces a parent by an
// ancestor), so every chain of reads strictly decreases and ends within N
// hops; `bound` (N + 1) only guards the kernel's exit. While links are being
// made, finds read device-coherently and halve the paths they walk (non-root
// entries only, so the compare-and-swap on roots is unaffected); afterwards
// the links are final and cached reads suffice.
template <bool LINKING>
__device__ __forceinline__ int32_t find_root(int32_t* par, int32_t x, int64_t bound) {
  constexpr int kScope = LINKING ? __HIP_MEMORY_SCOPE_AGENT : __HIP_MEMORY_SCOPE_WORKGROUP;
  for (int64_t i = 0; i < bound; ++i) {
    const int32_t p = __hip_atomic_load(&par[x], __ATOMIC_RELAXED, kScope);
    if (p < 0) return -1;
    if (p == x) return x;
    if (LINKING) {
      const int32_t gp = __hip_atomic_load(&par[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (gp < 0) return -1;
      if (gp != p) __hip_atomic_store(&par[x], gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      x = gp;
    } else {
      x = p;
    }
  }
  return -1;
}

__device__ __forceinline__ bool unite(int32_t* par, int32_t a, int32_t b, int64_t bound) {
  for (int64_t i = 0; i < bound; ++i) {
    a = find_root<true>(par, a, bound);
    b = find_root<true>(par, b, bound);
    if (a < 0 || b < 0) return false;
    if (a == b) return true;
    if (a < b) {
      const int32_t t = a;
      a = b;
      b = t;
    }
    int32_t expected = a;  // link the larger root under the smaller one
    if (__hip_atomic_compare_exchange_strong(&par[a], &expected, b, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT))
      return true;
    if (expected < 0 || expected >= a) return false;
    a = expected;  // a was linked meanwhile: continue from its parent
  }
  return false;
}

// Per-wave running sums for one key at a time (all lanes hold the same
// state): consecutive cells mostly belong to one bubble, so a wave walking a
// stretch of cells issues one atomic per change of key, not one per cell.
// Adds x to the order-free total (hi[k], lo[k]) (see fix_value).
__device__ __forceinline__ void fix_add(int64_t* hi, uint64_t* lo, int64_t k, double x) {
  if (!(fabs(x) < 0x1p62)) x = 0.0;  // (NaN only in a run already flagged unstable)
  double h = floor(x);
  double f = (x - h) * 0x1p64;
  if (!(f < 0x1p64)) {  // (a fraction within 2^-64 of 1)
    h += 1.0;
    f = 0.0;
  }
  const uint64_t l = (uint64_t)f;
  const uint64_t old = atomicAdd(reinterpret_cast<unsigned long long*>(&lo[k]), (unsigned long long)l);
  const int64_t carry = old + l < old ? 1 : 0;
  atomicAdd(reinterpret_cast<unsigned long long*>(&hi[k]), (unsigned long long)((int64_t)h + carry));
}

__device__ __forceinline__ double fix_get(const int64_t* hi, const uint64_t* lo, int64_t k) {
  return fix_value(hi[k], lo[k]);
}

// A wave's running sum for one key, flushed into an order-free total when
// the key changes (the wave's own additions come in a fixed order).
struct WaveSum {
  int32_t key = -1;
  double sum = 0.0;
  __device__ __forceinline__ void flush(int64_t* hi, uint64_t* lo) {
    if (key >= 0 && (threadIdx.x & 63) == 0) fix_add(hi, lo, key, sum);
    key = -1;
    sum = 0.0;
  }
  __device__ __forceinline__ void add(int64_t* hi, uint64_t* lo, int32_t k, double x) {
    if (k != key) {
      flush(hi, lo);
      key = k;
    }
    sum += x;
  }
};
struct WaveMin {
  int32_t key = -1, val = INT32_MAX;
  __device__ __forceinline__ void flush(int32_t* base) {
    if (key >= 0 && (threadIdx.x & 63) == 0) atomicMin(&base[key], val);
    key = -1;
    val = INT32_MAX;
  }
  __device__ __forceinline__ void add(int32_t* base, int32_t k, int32_t v) {
    if (k != key) {
      flush(base);
      key = k;
    }
    val = min(val, v);
  }
};

// Sum of v over the wave's active lanes of each distinct key, handed to acc.
__device__ __forceinline__ void wave_add(WaveSum& acc, int64_t* hi, uint64_t* lo, int32_t key, double v,
                                         bool act) {
  const int lane = threadIdx.x & 63;
  unsigned long long pending = __ballot(act);
  while (pending) {
    const int leader = __ffsll((long long)pending) - 1;
    const int32_t k = __shfl(key, leader);
    const bool mine = ((pending >> lane) & 1ull) && key == k;
    const unsigned long long m = __ballot(mine);
    double x = mine ? v : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    acc.add(hi, lo, k, x);
    pending &= ~m;
  }
}

// Smallest v over the wave's active lanes of each distinct key, handed to acc.
__device__ __forceinline__ void wave_min(WaveMin& acc, int32_t* base, int32_t key, int32_t v, bool act) {
  const int lane = threadIdx.x & 63;
  unsigned long long pending = __ballot(act);
  while (pending) {
    const int leader = __ffsll((long long)pending) - 1;
    const int32_t k = __shfl(key, leader);
    const bool mine = ((pending >> lane) & 1ull) && key == k;
    const unsigned long long m = __ballot(mine);
    int32_t x = mine ? v : INT32_MAX;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = min(x, __shfl_xor(x, o));
    acc.add(base, k, x);
    pending &= ~m;
  }
}

// Whether the bubbles must be found again: a step without marks changed no
// cell type, so its bubbles are the previous ones (labels already roots).
__device__ __forceinline__ bool bub_relabel(const Dev& d, int force) {
  return force || d.cnt[CNT_MARK0 + (d.step & 1)] != 0;
}

// Initial parents: within each wave's 64 consecutive cells, a bubble cell
// points at the first cell of its run of bubble cells along x (same row), so
// those links need no union; the runs are joined by the union pass. Without
// a relabelling the parents are the current labels.
// (Each pass is a body taking the block index, launched over one run by
// the k_bub_* kernels and over many by the batched ones.)
__device__ __forceinline__ void bub_init_body(const Dev& d, int blk, int force) {
  const int64_t c = (int64_t)blk * kBlock + threadIdx.x;
  // the per-bubble totals are kept at bubble roots: only bubble cells (the
  // new roots are among them) and the old roots (their label is their own
  // index) need clearing; the other entries are never read
  if (!bub_relabel(d, force)) {
    if (c >= d.g.N) return;
    const int32_t lab = d.blab[c];
    d.bpar[c] = lab;
    if (lab >= 0) {
      d.bV[c] = d.bW[c] = d.bR[c] = d.bnn[c] = 0;
      d.bVl[c] = d.bWl[c] = d.bRl[c] = d.bnnl[c] = 0;
    }
    d.bhas[c] = 0;
    d.btgt[c] = INT32_MAX;
    return;
  }
  const bool in = c < d.g.N;
  const bool bub = in && bubble_cell(d.flags[c]);
  const int lane = threadIdx.x & 63;
  const int x = in ? (int)(c % d.g.nx) : 0;
  const unsigned long long bm = __ballot(bub);
  const bool cont = bub && lane > 0 && x > 0 && ((bm >> (lane - 1)) & 1ull);
  const unsigned long long starts = bm & ~__ballot(cont);
  const unsigned long long upto = starts & (lane == 63 ? ~0ull : ((2ull << lane) - 1ull));
  const int first = upto ? 63 - __clzll((long long)upto) : lane;  // a bubble lane always has one
  if (!in) return;
  d.bpar[c] = bub ? (int32_t)(c - (lane - first)) : -1;
  if (bub || d.blab[c] == (int32_t)c) {
    d.bV[c] = d.bW[c] = d.bR[c] = d.bnn[c] = 0;
    d.bVl[c] = d.bWl[c] = d.bRl[c] = d.bnnl[c] = 0;
  }
  d.bhas[c] = 0;
  d.btgt[c] = INT32_MAX;
}

template <int Q>
__device__ __forceinline__ void bub_union_body(const Dev& d, int blk, int force) {
  if (!bub_relabel(d, force)) return;
  const int64_t c = (int64_t)blk * kBlock + threadIdx.x;
  if (c >= d.g.N || !bubble_cell(d.flags[c])) return;
  int x, y, z;
  coords(d.g, c, x, y, z);
  const int nx = d.g.nx;
  const int64_t bound = d.g.N + 1;
  bool ok = true;
  // +x: runs inside a wave's cells are joined by the initial parents; the
  // link across a wave boundary and across a periodic x face are made here
  {
    int w;
    const int64_t j = nb_index(d.g, x, y, z, 1, 0, 0, &w);
    if (j >= 0 && j != c && bubble_cell(d.flags[j]) && (x == nx - 1 || ((c + 1) & 63) == 0))
      ok &= unite(d.bpar, (int32_t)c, (int32_t)j, bound);
  }
  // the other directions, one of each opposite pair (every link seen from
  // one end); the link (c, j) is implied by (c - 1, j - 1) when c - 1 and
  // j - 1 are bubble cells beside c and j in their rows (x-linked to them)
  const bool left = x > 0 && bubble_cell(d.flags[c - 1]);
  for (int k = 3; k < Q; k += 2) {
    const int cx = cxd(k);
    int w;
    const int64_t j = nb_index(d.g, x, y, z, cx, cyd(k), czd(k), &w);
    if (j < 0 || j == c || !bubble_cell(d.flags[j])) continue;
    const int xj = x + cx;
    if (left && xj >= 1 && xj <= nx - 1 && bubble_cell(d.flags[j - 1])) continue;
    // an edge-diagonal link c + a + b (a, b two face steps) is implied by the
    // face links through c + a or c + b when either is a bubble cell
    const int cy = cyd(k), cz = czd(k);
    if ((cx != 0) + (cy != 0) + (cz != 0) == 2) {
      const int ax = cx != 0 ? cx : 0, ay = cx != 0 ? 0 : cy, az = cx != 0 || cy != 0 ? 0 : cz;
      int w1, w2;
      const int64_t m1 = nb_index(d.g, x, y, z, ax, ay, az, &w1);
      const int64_t m2 = nb_index(d.g, x, y, z, cx - ax, cy - ay, cz - az, &w2);
      if ((m1 >= 0 && bubble_cell(d.flags[m1])) || (m2 >= 0 && bubble_cell(d.flags[m2]))) continue;
    }
    // already joined as far as cached reads show (they see ancestors only)
    if (find_root<false>(d.bpar, (int32_t)c, bound) == find_root<false>(d.bpar, (int32_t)j, bound))
      continue;
    ok &= unite(d.bpar, (int32_t)c, (int32_t)j, bound);
  }
  if (!ok) atomicOr(&d.cnt[CNT_ERR], ERR_BUBBLE);
}

// Flattens the new labels; sums the new bubbles' volumes and the old
// bubbles' still-gaseous volumes. Each wave walks kBubIters stretches of 64
// cells (fewer atomics on the few addresses of large bubbles; few enough
// stretches that the walk's dependent reads stay short).
constexpr int kBubIters = 4;
__device__ __forceinline__ void bub_volume_body(const Dev& d, int blk) {
  const int lane = threadIdx.x & 63;
  const int64_t base = ((int64_t)blk * (kBlock / 64) + (threadIdx.x >> 6)) * 64 * kBubIters;
  WaveSum aV, aW;
  WaveMin aT;
  for (int it = 0; it < kBubIters; ++it) {
    const int64_t c = base + it * 64 + lane;
    const bool in = c < d.g.N;
    const uint8_t f = in ? d.flags[c] : 0;
    const bool bub = in && bubble_cell(f);
    int32_t r = -1;
    if (bub) {
      r = find_root<false>(d.bpar, (int32_t)c, d.g.N + 1);
      if (r < 0) atomicOr(&d.cnt[CNT_ERR], ERR_BUBBLE);
    }
    const bool ok = bub && r >= 0;
    const double w = ok ? ((f & T_MASK) == T_GAS ? 1.0 : 1.0 - d.phiB[c]) : 0.0;
    const int32_t old = ok ? d.blab[c] : -1;
    wave_add(aV, d.bV, d.bVl, r, w, ok);
    wave_add(aW, d.bW, d.bWl, old, w, old >= 0);
    wave_min(aT, d.btgt, old, r, old >= 0);
    // a root stays its own parent and r is an ancestor of c, so other
    // threads' finds through c still end at the same root
    if (ok) __hip_atomic_store(&d.bpar[c], r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  aV.flush(d.bV, d.bVl);
  aW.flush(d.bW, d.bWl);
  aT.flush(d.btgt);
}

// Amounts handed from old to new bubbles through the cells they share.
__device__ __forceinline__ void bub_amount_body(const Dev& d, int blk) {
  const int lane = threadIdx.x & 63;
  const int64_t base = ((int64_t)blk * (kBlock / 64) + (threadIdx.x >> 6)) * 64 * kBubIters;
  WaveSum aN, aR;
  for (int it = 0; it < kBubIters; ++it) {
    const int64_t c = base + it * 64 + lane;
    const bool in = c < d.g.N;
    const uint8_t f = in ? d.flags[c] : 0;
    const int32_t r = in && bubble_cell(f) ? d.bpar[c] : -1;
    const int32_t old = r >= 0 ? d.blab[c] : -1;
    double share = 0.0, w = 0.0;
    bool act = false;
    if (old >= 0) {
      const double W = fix_get(d.bW, d.bWl, old);
      if (W > 0.0) {
        d.bhas[r] = 1;
        if (r != d.btgt[old]) {
          w = (f & T_MASK) == T_GAS ? 1.0 : 1.0 - d.phiB[c];
          share = d.bamt[old] * (w / W);
          act = true;
        }
      }
    }
    wave_add(aN, d.bnn, d.bnnl, r, share, act);
    wave_add(aR, d.bR, d.bRl, old, w, act);
  }
  aN.flush(d.bnn, d.bnnl);
  aR.flush(d.bR, d.bRl);
}

// Each old bubble's target receives the rest of its amount.
__device__ __forceinline__ void bub_target_body(const Dev& d, int blk) {
  const int64_t c = (int64_t)blk * kBlock + threadIdx.x;
  if (c >= d.g.N) return;
  const int32_t t = d.btgt[c];
  if (t == INT32_MAX) return;  // (not an old bubble's root)
  const double W = fix_get(d.bW, d.bWl, c);
  if (!(W > 0.0)) return;
  fix_add(d.bnn, d.bnnl, t, d.bamt[c] * (1.0 - fix_get(d.bR, d.bRl, c) / W));
}

// Amount and pressure of each new bubble, at its root.
__device__ __forceinline__ void bub_pressure_body(const Dev& d, int blk) {
  const int64_t c = (int64_t)blk * kBlock + threadIdx.x;
  if (c >= d.g.N || d.bpar[c] != (int32_t)c) return;
  const double p0 = d.pV[1], V = fix_get(d.bV, d.bVl, c);
  const double n = d.bhas[c] ? fix_get(d.bnn, d.bnnl, c) : p0 * V;
  d.bamt[c] = n;
  d.bpr[c] = V > 0.0 ? n / V : p0;
}

// New labels become the current ones; gas density of every bubble cell from
// its bubble's pressure (interface cells read it in the next step; with
// surface tension the curvature pass adds the Laplace term).
__device__ __forceinline__ void bub_cells_body(const Dev& d, int blk) {
  const int64_t c = (int64_t)blk * kBlock + threadIdx.x;
  if (c >= d.g.N) return;
  const int32_t r = bubble_cell(d.flags[c]) ? d.bpar[c] : -1;
  d.blab[c] = r;
  if (r >= 0) d.rhoG[c] = 3.0 * d.bpr[r];
}

__global__ __launch_bounds__(kBlock) void k_bub_init(Dev d, int force) { bub_init_body(d, (int)blockIdx.x, force); }
template <int Q>
__global__ __launch_bounds__(kBlock) void k_bub_union(Dev d, int force) {
  bub_union_body<Q>(d, (int)blockIdx.x, force);
}
__global__ __launch_bounds__(kBlock) void k_bub_volume(Dev d) { bub_volume_body(d, (int)blockIdx.x); }
__global__ __launch_bounds__(kBlock) void k_bub_amount(Dev d) { bub_amount_body(d, (int)blockIdx.x); }
__global__ __launch_bounds__(kBlock) void k_bub_target(Dev d) { bub_target_body(d, (int)blockIdx.x); }
__global__ __launch_bounds__(kBlock) void k_bub_pressure(Dev d) { bub_pressure_body(d, (int)blockIdx.x); }
__global__ __launch_bounds__(kBlock) void k_bub_cells(Dev d) { bub_cells_body(d, (int)blockIdx.x); }

// grid of the volume and amount passes (kBubIters stretches of 64 cells per wave)
__host__ __device__ inline int64_t bub_walk_blocks(int64_t n) {
  return (n + kBlock * kBubIters - 1) / (kBlock * kBubIters);
}

#endif  // FSLBM_HOST_KERNELS

// ---------------------------------------------------------------------------
// Initialisation and export.
// ---------------------------------------------------------------------------
// types -> flags with the static BORDER bit; a liquid cell with a gas
// neighbour breaks the closed interface layer.
template <int Q>
__global__ __launch_bounds__(kBlock) void k_init_flags(Dev d) {
  const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const Geom& g = d.g;
  if (c >= g.N) return;
  const uint8_t t = d.flags[c];
  if (t > T_FREESLIP) {
    atomicOr(&d.cnt[CNT_ERR], ERR_TYPE);
    return;
  }
  int x, y, z;
  coords(g, c, x, y, z);
  bool border = (x == 0 || y == 0 || z == 0 || x == g.nx - 1 || y == g.ny - 1 || z == g.nz - 1);
  bool complex_ = false;
  bool gas_nb = false;
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int r[3] = {x + dx, y + dy, z + dz};
        const int n[3] = {g.nx, g.ny, g.nz};
        for (int a = 0; a < 3; ++a) {
          const int face = r[a] < 0 ? 2 * a : (r[a] >= n[a] ? 2 * a + 1 : -1);
          if (face >= 0 && face_kind(g, face) != BND_NOSLIP) complex_ = true;
        }
        int w;
        int64_t j = nb_index(g, x, y, z, dx, dy, dz, &w);
        if (j < 0) continue;
        const int tj = d.flags[j] & T_MASK;
        if (is_obst(tj)) border = complex_ = true;
      }
  for (int k = 1; k < Q; ++k) {
    int w;
    int64_t j = nb_index(g, x, y, z, cxd(k), cyd(k), czd(k), &w);
    if (j >= 0 && (d.flags[j] & T_MASK) == T_GAS) gas_nb = true;
  }
  if (t == T_LIQ && gas_nb) atomicOr(&d.cnt[CNT_ERR], ERR_LAYER);
  // the BORDER bit goes to a separate byte first (neighbours still read types)
  d.cls[c] = (uint8_t)((border ? F_BORDER : 0) | (complex_ ? F_COMPLEX | F_BORDER : 0));
}

#ifdef FSLBM_HOST_KERNELS
__global__ __launch_bounds__(kBlock) void k_apply_border(Dev d) {
  const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (c >= d.g.N) return;
  d.flags[c] = (uint8_t)((d.flags[c] & T_MASK) | d.cls[c]);
  d.cls[c] = CLS_STD;
}

#endif  // FSLBM_HOST_KERNELS

// Populations feq(rho, u) collided once; interface mass phi*rho; fill levels.
// On entry: rho in rho_if, u in (m, lost, phiB), phi in phiA. (At creation
// the step count is 0, where the in-place layout keeps f*_k(c) in plane k of
// c as the two-grid layout does.)
template <int S, int Q, bool TRT>
__global__ __launch_bounds__(kBlock) void k_init_state(Dev d, int resume) {
  using St = Store<S, Q>;
  using T = typename St::T;
  using R = typename St::R;
  const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const Geom& g = d.g;
  if (c >= g.N) return;
  const int t = d.flags[c] & T_MASK;
  T* A = static_cast<T*>(d.fA);
  double phi = d.phiA[c];
  if (t == T_LIQ) phi = 1.0;
  if (!is_fluid(t)) phi = 0.0;
  if (!resume) {
    const double rho = d.rho_if[c];
    const double ux = d.m[c], uy = d.lost[c], uz = d.phiB[c];
    if (is_fluid(t)) {
      R f[Q];
      const R usq = R(ux) * R(ux) + R(uy) * R(uy) + R(uz) * R(uz);
#pragma unroll
      for (int k = 0; k < Q; ++k)
        f[k] = feq_k<R, Q, St::kShift>(k, R(rho), R(rho - 1.0),
                                       cdot<R>(cxd(k), cyd(k), czd(k), R(ux), R(uy), R(uz)), usq);
      CollideParams<R> cp{R(d.omega), R(d.omega_m), R(d.gx), R(d.gy), R(d.gz), R(d.tau0), R(d.lambda), R(d.cs)};
      R rr, vx, vy, vz;
      collide<R, Q, TRT, St::kShift>(f, cp, rr, vx, vy, vz);
#pragma unroll
      for (int k = 0; k < Q; ++k) St::st(A, k * g.stride + c, k, f[k]);
    } else {
#pragma unroll
      for (int k = 0; k < Q; ++k) St::st(A, k * g.stride + c, k, R(0));
    }
  } else if (!is_fluid(t)) {
#pragma unroll
    for (int k = 0; k < Q; ++k) St::st(A, k * g.stride + c, k, R(0));
  }
  d.m[c] = (t == T_IF) ? phi * d.rho_if[c] : 0.0;
  d.phiA[c] = phi;
  d.phiB[c] = phi;
  d.lost[c] = 0.0;
  d.mark[c] = MK_NONE;
  d.rho_if[c] = 0.0;
}

// plane k of the resume populations (double) -> storage
template <int S, int Q>
__global__ __launch_bounds__(kBlock) void k_import_plane(Dev d, const double* src, int k) {
  using St = Store<S, Q>;
  const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (c >= d.g.N) return;
  const double v = St::kShift ? src[c] - weight<Q>(k) : src[c];
  St::st(static_cast<typename St::T*>(d.fA), k * d.g.stride + c, k, typename St::R(v));
}

// Export: what = 0 rho, 1 ux, 2 uy, 3 uz, 4 mass, 5 phi, 10 + k population plane k.
template <int S, int Q>
__global__ __launch_bounds__(kBlock) void k_export(Dev d, double* out, int what) {
  using St = Store<S, Q>;
  using T = typename St::T;
  using R = typename St::R;
  const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const Geom& g = d.g;
  if (c >= g.N) return;
  const T* A = static_cast<const T*>(d.fA);
  const uint8_t fb = d.flags[c];
  const int t = fb & T_MASK;
  const bool fl = is_fluid(t);
  const int par = (int)(d.step & 1);
  if (what >= 10) {
    const int k = what - 10;
    const double v = fl ? (double)St::ld(A, own_slot<Q>(d, c, fb, k, par), k) : 0.0;
    out[c] = fl ? (St::kShift ? weight<Q>(k) + v : v) : 0.0;
    return;
  }
  if (what == 5) {
    out[c] = d.phiA[c];
    return;
  }
  double v = 0.0;
  if (fl) {
    if (what == 4 && t == T_IF) {
      v = d.m[c];
    } else {
      R f[Q];
      if (d.aa && par) {
#pragma unroll
        for (int k = 0; k < Q; ++k) f[k] = St::ld(A, own_slot<Q>(d, c, fb, k, par), k);
      } else {
#pragma unroll
        for (int k = 0; k < Q; ++k) f[k] = St::ld(A, k * g.stride + c, k);
      }
      R rho, ux, uy, uz;
      post_moments<R, Q, St::kShift>(f, R(d.gx), R(d.gy), R(d.gz), rho, ux, uy, uz);
      v = what == 0 || what == 4 ? density64<R, Q, St::kShift>(f)
                                 : (what == 1 ? (double)ux : (what == 2 ? (double)uy : (double)uz));
    }
  }
  out[c] = v;
}

}  // namespace fslbm
