// HIP kernels of the free-surface LBM step for gfx950.
//
// One time step is four launches (plus two for surface tension, two for the
// bubble volume):
//   k_liquid    every liquid cell : pull streaming with walls, collision, store
//                                   (the bandwidth kernel)
//   k_interface list-driven       : every interface cell of the compacted list -
//                                   streaming, free-surface condition with the
//                                   variant's set, mass exchange, fill level,
//                                   conversion mark, collision
//   k_convert  every cell         : new type from the marks (to-gas marks next to
//                                   a to-liquid mark are dropped), in place; the
//                                   new interface list and the converted list are
//                                   compacted in ascending order by a single-pass
//                                   scan (wave ballot + decoupled look-back)
//   k_finish   list-driven        : reinitialise new interface cells from gas,
//                                   mass of new interface cells from liquid,
//                                   excess-mass gather, fill levels, flux classes
// The state between steps is the post-collision population f* (grid A); the
// step writes grid B and the host swaps A/B. Marks, counters and lists stay on the
// device, so a step needs no host synchronisation.
#pragma once

#include "fslbm_device.h"

namespace fslbm {

constexpr int kBlock = 256;

struct Dev {
  Geom g;
  // parameters
  double omega, omega_m, gx, gy, gz;
  double rho_gas, sigma, eps, delta;
  int variant, thurey, bubble;
  // state
  void* fA;  // post-collision populations at t (read)
  void* fB;  // post-collision populations at t+1 (written)
  uint8_t* flags;
  uint8_t* mark;
  uint8_t* cls;
  double* phiA;  // fill level at t (valid for every cell)
  double* phiB;  // fill level at t+1
  double* m;     // interface mass
  double* rho_if;
  double* rhoG;  // per-cell gas density (surface tension), or null
  double* phis;  // smoothed fill level (surface tension), or null
  double* lost;  // per-cell lost excess mass
  int32_t* if_list;
  int32_t* conv_list;
  int32_t* chunk_list;  // 64-cell chunks with liquid cells, ascending
  int32_t* cnt;
  unsigned long long* scan_if;
  unsigned long long* scan_cv;
  unsigned long long* scan_ch;
  double* pV;  // device scalars: [0] p^V, [1] p^V(0), [2] V(0)
  double* partial;  // reduction partials
  int64_t step;  // parity selects the mark-counter slot
};

// ---------------------------------------------------------------------------
// k_liquid and k_interface
// ---------------------------------------------------------------------------
template <int S, int Q>
__device__ __forceinline__ void load_plain(const typename Store<S, Q>::T* A, int64_t stride,
                                           int64_t c, int nx, int64_t nxy,
                                           typename Store<S, Q>::R* f) {
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    const int64_t off = kCX[k] + (int64_t)kCY[k] * nx + (int64_t)kCZ[k] * nxy;
    f[k] = Store<S, Q>::ld(A, k * stride + c - off, k);
  }
}

template <typename R>
__device__ __forceinline__ bool unstable(R rho, R ux, R uy, R uz) {
  const R usq = ux * ux + uy * uy + uz * uz;
  return !(rho > R(0)) || !(usq < R(1.0 / 3.0)) || !(rho == rho) || !(usq == usq) ||
         rho > R(1e30);
}

template <int S, int Q, bool TRT>
__device__ __forceinline__ void liquid_cell(const Dev& d, int64_t c) {
  using St = Store<S, Q>;
  using T = typename St::T;
  using R = typename St::R;
  const uint8_t fl = d.flags[c];
  if ((fl & T_MASK) != T_LIQ) return;
  const T* A = static_cast<const T*>(d.fA);
  T* B = static_cast<T*>(d.fB);
  const Geom& g = d.g;
  const int64_t stride = g.stride;
  R f[Q];
  if (!(fl & F_BORDER)) {
    load_plain<S, Q>(A, stride, c, g.nx, (int64_t)g.nx * g.ny, f);
  } else {
    int x, y, z;
    coords(g, c, x, y, z);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      int64_t src;
      int dir;
      bool wall;
      int kind = resolve_source<Q>(g, d.flags, x, y, z, k, &src, &dir, &wall);
      if (kind == SRC_FLUID) {
        f[k] = St::ld(A, dir * stride + src, dir);
      } else {
        if (kind == SRC_GAS) atomicOr(&d.cnt[CNT_ERR], ERR_LAYER);
        f[k] = St::ld(A, opp(k) * stride + c, opp(k));
      }
    }
  }
  CollideParams<R> cp{R(d.omega), R(d.omega_m), R(d.gx), R(d.gy), R(d.gz)};
  R rho, ux, uy, uz;
  collide<R, Q, TRT, St::kShift>(f, cp, rho, ux, uy, uz);
  if (unstable(rho, ux, uy, uz)) atomicOr(&d.cnt[CNT_ERR], ERR_UNSTABLE);
#pragma unroll
  for (int k = 0; k < Q; ++k) St::st(B, k * stride + c, k, f[k]);
}

// Parker-Youngs normal n = grad(phi) (Sec. 2.2) over the 3x3x3 neighbourhood;
// obstacle points take the centre value.
__device__ __forceinline__ void py_normal(const Geom& g, const uint8_t* flags, const double* phi,
                                          int x, int y, int z, double v0, double n[3]) {
  const double W[3] = {1.0, 2.0, 1.0};
#pragma unroll 1
  for (int a = 0; a < 3; ++a) {
    const int a1 = (a + 1) % 3, a2 = (a + 2) % 3;
    double s = 0.0;
#pragma unroll 1
    for (int b = -1; b <= 1; ++b) {
#pragma unroll 1
      for (int cc = -1; cc <= 1; ++cc) {
        int dp[3], dm[3];
        dp[a] = 1;
        dm[a] = -1;
        dp[a1] = dm[a1] = b;
        dp[a2] = dm[a2] = cc;
        int64_t ip, im;
        int tp = nb_type(g, flags, x, y, z, dp[0], dp[1], dp[2], &ip);
        int tm = nb_type(g, flags, x, y, z, dm[0], dm[1], dm[2], &im);
        double vp = is_obst(tp) ? v0 : phi[ip];
        double vm = is_obst(tm) ? v0 : phi[im];
        s += W[b + 1] * W[cc + 1] * (vp - vm);
      }
    }
    n[a] = s;
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

template <int S, int Q, bool TRT>
__device__ __forceinline__ void interface_cell(const Dev& d, int64_t c) {
  using St = Store<S, Q>;
  using T = typename St::T;
  using R = typename St::R;
  const T* A = static_cast<const T*>(d.fA);
  T* B = static_cast<T*>(d.fB);
  const Geom& g = d.g;
  const int64_t stride = g.stride;
  int x, y, z;
  coords(g, c, x, y, z);

  // own post-collision populations and the velocity of the collision at t
  R fo[Q];
#pragma unroll
  for (int k = 0; k < Q; ++k) fo[k] = St::ld(A, k * stride + c, k);
  R rho_t, ux, uy, uz;
  constexpr bool SH = St::kShift;
  post_moments<R, Q, SH>(fo, R(d.gx), R(d.gy), R(d.gz), rho_t, ux, uy, uz);
  const R usq = ux * ux + uy * uy + uz * uz;

  // missing populations: direct gas sources
  uint32_t gas = 0;
#pragma unroll
  for (int k = 1; k < Q; ++k) {
    int64_t j;
    if (nb_type(g, d.flags, x, y, z, -kCX[k], -kCY[k], -kCZ[k], &j) == T_GAS) gas |= 1u << k;
  }
  const int missing = __builtin_popcount(gas);

  // the variant's reconstruction set (Sec. 3)
  uint32_t R_set = gas;
  const int v = d.variant;
  const bool nb_based = (v == 1 || v == 2 || (v == 4 && missing < 3));
  const double phi_c = d.phiA[c];
  if (nb_based) {
    double n[3];
    py_normal(g, d.flags, d.phiA, x, y, z, phi_c, n);
    double nmax = fabs(n[0]);
    nmax = fabs(n[1]) > nmax ? fabs(n[1]) : nmax;
    nmax = fabs(n[2]) > nmax ? fabs(n[2]) : nmax;
    const double thr = -d.delta * nmax;
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      if (k == 0 && v != 1) continue;
      const double dot = n[0] * kCX[k] + n[1] * kCY[k] + n[2] * kCZ[k];
      if (dot >= thr) R_set |= 1u << k;
    }
  }

  const R rhoG = d.rhoG ? R(d.rhoG[c]) : R(d.pV[0] * 3.0);
  const int cls_c = d.cls[c];

  // streaming, boundary condition and mass exchange (Sec. 2.2)
  R f[Q];
  double dm = 0.0;
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    int64_t src;
    int dir;
    bool wall;
    const int kind = resolve_source<Q>(g, d.flags, x, y, z, k, &src, &dir, &wall);
    R in_val = R(0);
    if (kind == SRC_FLUID) in_val = St::ld(A, dir * stride + src, dir);
    if (kind == SRC_BOUNCE) {
      f[k] = fo[opp(k)];
    } else if (kind == SRC_GAS || (((R_set >> k) & 1u) && !wall)) {
      f[k] = abb_value<R, Q, SH>(k, rhoG, ux, uy, uz, usq, fo[opp(k)]);
    } else {
      f[k] = in_val;
    }
    if (k > 0 && kind == SRC_FLUID) {
      const double in = (double)in_val, out = (double)fo[opp(k)];
      const uint8_t ts = d.flags[src] & T_MASK;
      if (ts == T_LIQ) {
        dm += in - out;
      } else {
        const double T_ = d.thurey ? flux_term(cls_c, d.cls[src], in, out) : in - out;
        dm += 0.5 * (phi_c + d.phiA[src]) * T_;
      }
    }
  }

  // fill level and conversion mark
  const double rho_n = density64<R, Q, SH>(f);
  const double m_new = d.m[c] + dm;
  const double phi_n = m_new / rho_n;
  uint8_t mk = MK_NONE;
  if (phi_n > 1.0 + d.eps)
    mk = MK_L;
  else if (phi_n < -d.eps)
    mk = MK_G;
  d.m[c] = m_new;
  d.rho_if[c] = rho_n;
  d.phiB[c] = phi_n;
  d.mark[c] = mk;
  if (mk) atomicAdd(&d.cnt[CNT_MARK0 + (d.step & 1)], 1);

  CollideParams<R> cp{R(d.omega), R(d.omega_m), R(d.gx), R(d.gy), R(d.gz)};
  R rho, vx, vy, vz;
  collide<R, Q, TRT, SH>(f, cp, rho, vx, vy, vz);
  if (unstable(rho, vx, vy, vz) || !(m_new == m_new)) atomicOr(&d.cnt[CNT_ERR], ERR_UNSTABLE);
#pragma unroll
  for (int k = 0; k < Q; ++k) St::st(B, k * stride + c, k, f[k]);
}

// Each wave takes 64-cell chunks from the chunk list (chunks without liquid
// cells are never visited), one cell per lane.
template <int S, int Q, bool TRT>
__global__ __launch_bounds__(kBlock) void k_liquid(Dev d) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    d.cnt[CNT_MARK0 + ((d.step + 1) & 1)] = 0;  // slot of the next step
    d.cnt[CNT_TICKET] = 0;
    d.cnt[CNT_EPOCH] += 1;  // a new epoch for this step's compaction scan
  }
  const int nch = d.cnt[CNT_CHUNKS];
  const int lane = threadIdx.x & 63;
  const int waves = gridDim.x * (kBlock / 64);
  for (int w = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); w < nch; w += waves) {
    const int64_t c = (int64_t)d.chunk_list[w] * 64 + lane;
    if (c < d.g.N) liquid_cell<S, Q, TRT>(d, c);
  }
}

template <int S, int Q, bool TRT>
__global__ __launch_bounds__(kBlock) void k_interface(Dev d) {
  const int nif = d.cnt[CNT_IF];
  for (int k = blockIdx.x * kBlock + threadIdx.x; k < nif; k += gridDim.x * kBlock)
    interface_cell<S, Q, TRT>(d, d.if_list[k]);
}

// ---------------------------------------------------------------------------
// k_convert: new types from marks, in place, plus compaction.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool any_nb_mark(const Dev& d, int x, int y, int z, int64_t c,
                                            bool border, int Q, uint8_t want) {
  const Geom& g = d.g;
  const int64_t nx = g.nx, nxy = (int64_t)g.nx * g.ny;
  for (int k = 1; k < Q; ++k) {
    int64_t j;
    if (!border) {
      j = c + kCX[k] + kCY[k] * nx + kCZ[k] * nxy;
    } else {
      int w;
      j = nb_index(g, x, y, z, kCX[k], kCY[k], kCZ[k], &w);
      if (j < 0) continue;
    }
    if (d.mark[j] == want) return true;
  }
  return false;
}

// A to-gas mark survives unless a to-liquid mark is in its neighbourhood
// (Sec. 2.2: separation of liquid and gas has priority).
__device__ __forceinline__ bool gas_mark_kept(const Dev& d, int64_t j, int Q) {
  if (d.mark[j] != MK_G) return false;
  int x, y, z;
  coords(d.g, j, x, y, z);
  return !any_nb_mark(d, x, y, z, j, (d.flags[j] & F_BORDER) != 0, Q, MK_L);
}

__device__ __forceinline__ unsigned long long pack_status(uint32_t epoch, uint32_t flag,
                                                          uint32_t val) {
  return ((unsigned long long)epoch << 32) | ((unsigned long long)flag << 30) | val;
}

// Exclusive prefix of this tile's aggregate over all earlier tiles, computed by
// one wave with decoupled look-back: each tile publishes its aggregate (flag 1)
// at once and its inclusive prefix (flag 2) when known; a tile sums the
// aggregates of its predecessors back to the nearest inclusive prefix, 64 tiles
// per round. Entries carry the launch epoch, so the array never needs clearing.
// The status word is the only datum exchanged, so relaxed device-scope atomics
// suffice (no acquire/release: those would flush the XCD's L2 on every poll).
// The wait on a predecessor is bounded: on expiry the scan error bit is set and
// the kernel completes (with a wrong list, reported by the host).
__device__ uint32_t lookback_wave(unsigned long long* status, int tile, uint32_t agg,
                                  uint32_t epoch, int32_t* err) {
  const int lane = threadIdx.x & 63;
  if (lane == 0)
    __hip_atomic_store(&status[tile], pack_status(epoch, tile == 0 ? 2u : 1u, agg),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  uint32_t excl = 0;
  int base = tile - 1;
  bool done = (tile == 0);
  int spins = 0;
  while (!done) {
    const int t = base - lane;
    unsigned long long v = 0;
    uint32_t fl = 3u;  // before the first tile: acts as an inclusive prefix of 0
    if (t >= 0) {
      for (;;) {
        v = __hip_atomic_load(&status[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((uint32_t)(v >> 32) == epoch) break;
        if (++spins > (1 << 22)) {
          atomicOr(err, ERR_SCAN);
          v = pack_status(epoch, 2u, 0u);
          break;
        }
        if (spins > 64) __builtin_amdgcn_s_sleep(1);
      }
      fl = (uint32_t)(v >> 30) & 3u;
    }
    const uint32_t val = (t >= 0) ? (uint32_t)(v & 0x3fffffffu) : 0u;
    const unsigned long long pm = __ballot(fl >= 2u);
    const int stop = pm ? __builtin_ctzll(pm) : 64;
    uint32_t contrib = (lane <= stop) ? val : 0u;
    for (int o = 32; o > 0; o >>= 1) contrib += __shfl_xor(contrib, o, 64);
    excl += contrib;
    if (pm)
      done = true;
    else
      base -= 64;
  }
  if (lane == 0 && tile > 0)
    __hip_atomic_store(&status[tile], pack_status(epoch, 2u, excl + agg), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  return excl;
}

// New cell type of cell c from its flags and the marks around it.
template <int Q>
__device__ __forceinline__ uint8_t new_flags(const Dev& d, int64_t c, uint8_t fl) {
  const Geom& g = d.g;
  const int t = fl & T_MASK;
  int nt = t;
  uint8_t bits = 0;
  const bool border = (fl & F_BORDER) != 0;
  int x = 0, y = 0, z = 0;
  if (border) coords(g, c, x, y, z);
  if (t == T_IF) {
    const uint8_t mk = d.mark[c];
    if (mk == MK_L) {
      nt = T_LIQ;
      bits = F_CONV;
    } else if (mk == MK_G && !any_nb_mark(d, x, y, z, c, border, Q, MK_L)) {
      nt = T_GAS;
      bits = F_CONV;
    }
  } else if (t == T_GAS) {
    if (any_nb_mark(d, x, y, z, c, border, Q, MK_L)) {
      nt = T_IF;
      bits = F_NEW_GAS;
    }
  } else if (t == T_LIQ) {
    const int64_t nx = g.nx, nxy = (int64_t)g.nx * g.ny;
    for (int k = 1; k < Q; ++k) {
      int64_t j;
      if (!border) {
        j = c + kCX[k] + kCY[k] * nx + kCZ[k] * nxy;
      } else {
        int w;
        j = nb_index(g, x, y, z, kCX[k], kCY[k], kCZ[k], &w);
        if (j < 0) continue;
      }
      if (gas_mark_kept(d, j, Q)) {
        nt = T_IF;
        bits = F_NEW_LIQ;
        break;
      }
    }
  }
  return (uint8_t)((fl & F_BORDER) | nt | bits);
}

constexpr int kConvPer = 16;                   // cells per thread in k_convert
constexpr int kConvTile = kBlock * kConvPer;  // cells per tile

// One tile = kConvTile consecutive cells, slice j = cells [j*256, (j+1)*256) of
// the tile. List order inside a tile is slice-major, thread-minor, i.e.
// ascending cell index.
template <int Q>
__global__ __launch_bounds__(kBlock) void k_convert(Dev d, int rebuild_only) {
  if (!rebuild_only && d.cnt[CNT_MARK0 + (d.step & 1)] == 0) return;
  __shared__ int s_tile;
  __shared__ uint32_t s_wc[2][kConvPer][kBlock / 64];
  __shared__ uint8_t s_ch[kConvPer][kBlock / 64];
  __shared__ uint32_t s_excl[3];
  if (threadIdx.x == 0) s_tile = atomicAdd(&d.cnt[CNT_TICKET], 1);
  __syncthreads();
  const int tile = s_tile;
  const uint32_t epoch = (uint32_t)d.cnt[CNT_EPOCH];
  const int64_t base = (int64_t)tile * kConvTile;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint32_t pif = 0, pcv = 0;
  uint32_t rif[kConvPer], rcv[kConvPer];
#pragma unroll
  for (int j = 0; j < kConvPer; ++j) {
    const int64_t c = base + j * kBlock + threadIdx.x;
    bool is_if = false, is_cv = false, is_liq = false;
    if (c < d.g.N) {
      const uint8_t fl = d.flags[c];
      uint8_t nf = fl;
      if (!rebuild_only) {
        nf = new_flags<Q>(d, c, fl);
        if (nf != fl) d.flags[c] = nf;
      }
      is_if = (nf & T_MASK) == T_IF;
      is_liq = (nf & T_MASK) == T_LIQ;
      is_cv = (nf & F_CONV) != 0;
    }
    const bool chunk_active = __ballot(is_liq) != 0ull;
    pif |= (uint32_t)is_if << j;
    pcv |= (uint32_t)is_cv << j;
    const unsigned long long bi = __ballot(is_if), bc = __ballot(is_cv);
    rif[j] = __popcll(bi & below);
    rcv[j] = __popcll(bc & below);
    if (lane == 0) {
      s_wc[0][j][wv] = __popcll(bi);
      s_wc[1][j][wv] = __popcll(bc);
      s_ch[j][wv] = chunk_active;
    }
  }
  __syncthreads();
  // tile aggregates
  uint32_t agg[3] = {0, 0, 0};
#pragma unroll
  for (int j = 0; j < kConvPer; ++j)
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
      agg[0] += s_wc[0][j][w];
      agg[1] += s_wc[1][j][w];
      agg[2] += s_ch[j][w];
    }
  if (wv < 3) {
    unsigned long long* st = wv == 0 ? d.scan_if : (wv == 1 ? d.scan_cv : d.scan_ch);
    const uint32_t e = lookback_wave(st, tile, agg[wv], epoch, &d.cnt[CNT_ERR]);
    if (lane == 0) s_excl[wv] = e;
  }
  __syncthreads();
  // chunk list: one entry per active (slice, wave) pair, thread 0 writes them
  if (threadIdx.x == 0) {
    uint32_t o = s_excl[2];
    for (int j = 0; j < kConvPer; ++j)
      for (int w = 0; w < kBlock / 64; ++w)
        if (s_ch[j][w]) d.chunk_list[o++] = tile * (kConvTile / 64) + j * (kBlock / 64) + w;
    if (tile == (int)gridDim.x - 1) d.cnt[CNT_CHUNKS] = (int32_t)o;
  }
  uint32_t off[2] = {s_excl[0], s_excl[1]};
#pragma unroll
  for (int j = 0; j < kConvPer; ++j) {
    uint32_t wo0 = 0, wo1 = 0, t0 = 0, t1 = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
      if (w < wv) {
        wo0 += s_wc[0][j][w];
        wo1 += s_wc[1][j][w];
      }
      t0 += s_wc[0][j][w];
      t1 += s_wc[1][j][w];
    }
    const int64_t c = base + j * kBlock + threadIdx.x;
    if ((pif >> j) & 1u) d.if_list[off[0] + wo0 + rif[j]] = (int32_t)c;
    if ((pcv >> j) & 1u) d.conv_list[off[1] + wo1 + rcv[j]] = (int32_t)c;
    off[0] += t0;
    off[1] += t1;
  }
  if (tile == (int)gridDim.x - 1 && threadIdx.x == 0) {
    d.cnt[CNT_IF] = (int32_t)off[0];
    d.cnt[CNT_CONV] = (int32_t)off[1];
  }
}

// ---------------------------------------------------------------------------
// k_finish: list-driven completion of the conversion.
// ---------------------------------------------------------------------------
template <int Q>
__device__ __forceinline__ int count_if_nb(const Dev& d, int64_t z) {
  int x, y, zz;
  coords(d.g, z, x, y, zz);
  int n = 0;
  for (int k = 1; k < Q; ++k) {
    int w;
    int64_t j = nb_index(d.g, x, y, zz, kCX[k], kCY[k], kCZ[k], &w);
    if (j >= 0 && (d.flags[j] & T_MASK) == T_IF) ++n;
  }
  return n;
}

// Excess mass of a converted cell (Sec. 2.2): m - rho when filled, m when emptied.
__device__ __forceinline__ double excess_of(const Dev& d, int64_t z) {
  const int t = d.flags[z] & T_MASK;
  return t == T_LIQ ? d.m[z] - d.rho_if[z] : d.m[z];
}

template <int S, int Q, bool TRT>
__device__ void finish_interface(const Dev& d, int64_t c) {
  using St = Store<S, Q>;
  using T = typename St::T;
  using R = typename St::R;
  constexpr bool SH = St::kShift;
  T* B = static_cast<T*>(d.fB);
  const Geom& g = d.g;
  const int64_t stride = g.stride;
  const uint8_t fl = d.flags[c];
  int x, y, z;
  coords(g, c, x, y, z);
  double mass, rho_n;
  if (fl & F_NEW_GAS) {
    // equilibrium of the mean density and velocity of the liquid and old
    // interface neighbours (Sec. 2.2), then the collision of this step
    R rs = R(0), us0 = R(0), us1 = R(0), us2 = R(0);
    int cnt = 0;
    for (int k = 1; k < Q; ++k) {
      int w;
      int64_t j = nb_index(g, x, y, z, kCX[k], kCY[k], kCZ[k], &w);
      if (j < 0) continue;
      const uint8_t fj = d.flags[j];
      if (!is_fluid(fj & T_MASK) || (fj & F_NEW_GAS)) continue;
      R fj_[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) fj_[i] = St::ld(B, i * stride + j, i);
      R r, a, b, cc;
      post_moments<R, Q, SH>(fj_, R(d.gx), R(d.gy), R(d.gz), r, a, b, cc);
      rs += r;
      us0 += a;
      us1 += b;
      us2 += cc;
      cnt += 1;
    }
    const R rb = rs / R(cnt);
    const R ub0 = us0 / R(cnt), ub1 = us1 / R(cnt), ub2 = us2 / R(cnt);
    const R usq = ub0 * ub0 + ub1 * ub1 + ub2 * ub2;
    R f[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k)
      f[k] = feq_k<R, Q, SH>(k, rb, rb - R(1), cdot<R>(kCX[k], kCY[k], kCZ[k], ub0, ub1, ub2),
                             usq);
    CollideParams<R> cp{R(d.omega), R(d.omega_m), R(d.gx), R(d.gy), R(d.gz)};
    R rr, vx, vy, vz;
    collide<R, Q, TRT, SH>(f, cp, rr, vx, vy, vz);
#pragma unroll
    for (int k = 0; k < Q; ++k) St::st(B, k * stride + c, k, f[k]);
    mass = 0.0;
    rho_n = (double)rb;
  } else if (fl & F_NEW_LIQ) {
    R fc[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) fc[k] = St::ld(B, k * stride + c, k);
    const double r = density64<R, Q, SH>(fc);
    mass = r;
    rho_n = r;
  } else {
    mass = d.m[c];
    rho_n = d.rho_if[c];
  }
  // excess mass of converted neighbours, equal shares over their interface
  // neighbours, added in direction order
  bool has_liq = false, has_gas = false;
  for (int k = 1; k < Q; ++k) {
    int w;
    int64_t j = nb_index(g, x, y, z, kCX[k], kCY[k], kCZ[k], &w);
    if (j < 0) continue;
    const uint8_t fj = d.flags[j];
    const int tj = fj & T_MASK;
    has_liq |= (tj == T_LIQ);
    has_gas |= (tj == T_GAS);
    if (fj & F_CONV) mass += excess_of(d, j) / (double)count_if_nb<Q>(d, j);
  }
  d.m[c] = mass;
  d.rho_if[c] = rho_n;
  d.phiB[c] = mass / rho_n;
  d.cls[c] = (!has_liq && has_gas) ? CLS_NOLIQ : ((!has_gas && has_liq) ? CLS_NOGAS : CLS_STD);
}

template <int Q>
__device__ void finish_converted(const Dev& d, int64_t z) {
  const int t = d.flags[z] & T_MASK;
  if (count_if_nb<Q>(d, z) == 0) d.lost[z] += excess_of(d, z);
  d.mark[z] = MK_NONE;
  const double v = (t == T_LIQ) ? 1.0 : 0.0;
  d.phiA[z] = v;
  d.phiB[z] = v;
}

template <int S, int Q, bool TRT>
__global__ __launch_bounds__(kBlock) void k_finish(Dev d, int classes_only) {
  if (!classes_only && d.cnt[CNT_MARK0 + (d.step & 1)] == 0) return;
  const int nif = d.cnt[CNT_IF];
  const int ncv = classes_only ? 0 : d.cnt[CNT_CONV];
  const int total = nif + ncv;
  for (int k = blockIdx.x * kBlock + threadIdx.x; k < total; k += gridDim.x * kBlock) {
    if (k < nif) {
      const int64_t c = d.if_list[k];
      if (classes_only) {
        int x, y, z;
        coords(d.g, c, x, y, z);
        bool has_liq = false, has_gas = false;
        for (int i = 1; i < Q; ++i) {
          int w;
          int64_t j = nb_index(d.g, x, y, z, kCX[i], kCY[i], kCZ[i], &w);
          if (j < 0) continue;
          const int tj = d.flags[j] & T_MASK;
          has_liq |= (tj == T_LIQ);
          has_gas |= (tj == T_GAS);
        }
        d.cls[c] = (!has_liq && has_gas) ? CLS_NOLIQ : ((!has_gas && has_liq) ? CLS_NOGAS : CLS_STD);
      } else {
        finish_interface<S, Q, TRT>(d, c);
      }
    } else {
      finish_converted<Q>(d, d.conv_list[k - nif]);
    }
  }
}

// ---------------------------------------------------------------------------
// Surface tension (Sec. 2.2): K8-smoothed fill level, curvature, gas density.
// ---------------------------------------------------------------------------
#ifdef FSLBM_HOST_KERNELS
// Smoothed fill level of every cell, K(r) = (1 - r^2/4)^4 over the 3x3x3 box
// (support radius 2), obstacles left out and the weights renormalised. The
// block stages a (64+2) x (4+2) x (1+2) halo of phi and flags in LDS.
__global__ __launch_bounds__(kBlock) void k_smooth(Dev d) {
  constexpr int TX = 64, TY = 4;
  __shared__ double s_phi[3][TY + 2][TX + 2];
  __shared__ uint8_t s_obs[3][TY + 2][TX + 2];
  const Geom& g = d.g;
  const int tiles_x = (g.nx + TX - 1) / TX, tiles_y = (g.ny + TY - 1) / TY;
  const int bt = blockIdx.x;
  const int tz = bt / (tiles_x * tiles_y);
  const int r = bt - tz * tiles_x * tiles_y;
  const int ty0 = (r / tiles_x) * TY, tx0 = (r % tiles_x) * TX;
  for (int e = threadIdx.x; e < 3 * (TY + 2) * (TX + 2); e += kBlock) {
    const int lz = e / ((TY + 2) * (TX + 2));
    const int rr = e - lz * (TY + 2) * (TX + 2);
    const int ly = rr / (TX + 2), lx = rr - ly * (TX + 2);
    int w;
    const int64_t j = nb_index(g, tx0 + lx - 1, ty0 + ly - 1, tz + lz - 1, 0, 0, 0, &w);
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

__device__ __forceinline__ void unit_normal_s(const Dev& d, int64_t j, double nh[3]) {
  int x, y, z;
  coords(d.g, j, x, y, z);
  double n[3];
  py_normal(d.g, d.flags, d.phis, x, y, z, d.phis[j], n);
  const double len = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  if (len > 0.0) {
    nh[0] = n[0] / len;
    nh[1] = n[1] / len;
    nh[2] = n[2] / len;
  } else {
    nh[0] = nh[1] = nh[2] = 0.0;
  }
}

// kappa = -div(n_hat) by central differences of the unit normals of the face
// neighbours; rho^G = 3 (p^V + sigma kappa).
__global__ __launch_bounds__(kBlock) void k_curvature(Dev d) {
  const int nif = d.cnt[CNT_IF];
  for (int k = blockIdx.x * kBlock + threadIdx.x; k < nif; k += gridDim.x * kBlock) {
    const int64_t c = d.if_list[k];
    int x, y, z;
    coords(d.g, c, x, y, z);
    double nc[3];
    unit_normal_s(d, c, nc);
    double div = 0.0;
    for (int a = 0; a < 3; ++a) {
      int e[3] = {0, 0, 0};
      double np_, nm_;
      int w;
      e[a] = 1;
      int64_t jp = nb_index(d.g, x, y, z, e[0], e[1], e[2], &w);
      if (jp < 0 || is_obst(d.flags[jp] & T_MASK)) {
        np_ = nc[a];
      } else {
        double t[3];
        unit_normal_s(d, jp, t);
        np_ = t[a];
      }
      e[a] = -1;
      int64_t jm = nb_index(d.g, x, y, z, e[0], e[1], e[2], &w);
      if (jm < 0 || is_obst(d.flags[jm] & T_MASK)) {
        nm_ = nc[a];
      } else {
        double t[3];
        unit_normal_s(d, jm, t);
        nm_ = t[a];
      }
      div += 0.5 * (np_ - nm_);
    }
    const double kappa = -div;
    d.rhoG[c] = 3.0 * (d.pV[0] + d.sigma * kappa);
  }
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
    const int t = d.flags[c] & T_MASK;
    if (t == T_LIQ) {
      typename St::R f[Q];
#pragma unroll
      for (int k = 0; k < Q; ++k) f[k] = St::ld(A, k * d.g.stride + c, k);
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
__global__ __launch_bounds__(kBlock) void k_reduce_volume(Dev d, int cells_per_block) {
  double v[1] = {0.0};
  const int64_t begin = (int64_t)blockIdx.x * cells_per_block;
  int64_t end = begin + cells_per_block;
  if (end > d.g.N) end = d.g.N;
  for (int64_t c = begin + threadIdx.x; c < end; c += kBlock) {
    const int t = d.flags[c] & T_MASK;
    if (t == T_GAS)
      v[0] += 1.0;
    else if (t == T_IF)
      v[0] += 1.0 - d.phiB[c];
  }
  block_reduce_store<1>(v, d.partial + blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void k_sum_partials(const double* partial, int nblocks,
                                                         int nv, double* out) {
  // thread i sums value i over the partials in block order
  if ((int)threadIdx.x < nv) {
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += partial[(int64_t)b * nv + threadIdx.x];
    out[threadIdx.x] = s;
  }
}

__global__ void k_update_pv(double* pV, const double* V) {
  if (threadIdx.x == 0) pV[0] = pV[1] * pV[2] / V[0];
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
  bool gas_nb = false;
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        int w;
        int64_t j = nb_index(g, x, y, z, dx, dy, dz, &w);
        if (j < 0) continue;
        const int tj = d.flags[j] & T_MASK;
        if (is_obst(tj)) border = true;
      }
  for (int k = 1; k < Q; ++k) {
    int w;
    int64_t j = nb_index(g, x, y, z, kCX[k], kCY[k], kCZ[k], &w);
    if (j >= 0 && (d.flags[j] & T_MASK) == T_GAS) gas_nb = true;
  }
  if (t == T_LIQ && gas_nb) atomicOr(&d.cnt[CNT_ERR], ERR_LAYER);
  // the BORDER bit goes to a separate byte first (neighbours still read types)
  d.cls[c] = border ? F_BORDER : 0;
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
// On entry: rho in rho_if, u in (m, lost, phiB), phi in phiA.
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
                                       cdot<R>(kCX[k], kCY[k], kCZ[k], R(ux), R(uy), R(uz)), usq);
      CollideParams<R> cp{R(d.omega), R(d.omega_m), R(d.gx), R(d.gy), R(d.gz)};
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
  const int t = d.flags[c] & T_MASK;
  const bool fl = is_fluid(t);
  if (what >= 10) {
    const int k = what - 10;
    const double v = (double)St::ld(A, k * g.stride + c, k);
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
#pragma unroll
      for (int k = 0; k < Q; ++k) f[k] = St::ld(A, k * g.stride + c, k);
      R rho, ux, uy, uz;
      post_moments<R, Q, St::kShift>(f, R(d.gx), R(d.gy), R(d.gz), rho, ux, uy, uz);
      v = what == 0 || what == 4 ? density64<R, Q, St::kShift>(f) : (what == 1 ? (double)ux : (what == 2 ? (double)uy : (double)uz));
    }
  }
  out[c] = v;
}

}  // namespace fslbm
