// HIP kernels of the free-surface LBM step for gfx950.
//
// One time step is four launches (plus two for surface tension, two for the
// bubble volume):
//   k_liquid    chunk-list-driven : every liquid cell away from walls - pull
//                                   streaming, collision, store (the bandwidth
//                                   kernel)
//   k_generic   list-driven       : every interface cell of the compacted list -
//                                   streaming, free-surface condition with the
//                                   variant's set, mass exchange, fill level,
//                                   conversion mark, collision - and every liquid
//                                   cell next to a wall or obstacle
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
constexpr int kConvPer = 64;                   // cells per thread in k_convert (one chunk)
constexpr int kConvTile = kBlock * kConvPer;  // cells per compaction tile

struct Dev {
  Geom g;
  // parameters
  double omega, omega_m, gx, gy, gz;
  double tau0, lambda, cs;  // Smagorinsky model (cs = 0: off)
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
  int32_t* gen_list;    // liquid cells with the BORDER flag, ascending
  uint8_t* tile_dirty;  // per compaction tile: a conversion mark lies in or next to it
  uint8_t* cand;        // per cell: lies in the 3x3x3 neighbourhood of a marked cell
  int32_t* cnt;
  unsigned long long* scan_if;
  unsigned long long* scan_cv;
  unsigned long long* scan_ch;
  unsigned long long* scan_gen;
  double* pV;  // device scalars: [0] p^V, [1] p^V(0), [2] V(0)
  double* partial;  // reduction partials
  int64_t step;  // parity selects the mark-counter slot
};

// ---------------------------------------------------------------------------
// k_liquid and k_generic
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

// Liquid cell without the COMPLEX flag: pull from the linear neighbour
// offsets, or - for a cell on a no-slip domain face - bounce-back of its own
// opposite population where the source lies beyond the face; collision; store.
// (A liquid cell never has a gas neighbour, so no free-surface logic applies.)
// BUF: both grids fit a 32-bit byte range, so loads and stores go through
// buffer resources; inside the domain a wave uses one per-lane offset (the
// cell) plus a scalar offset per direction (plane start minus the neighbour
// offset).
template <int S, int Q, bool TRT, bool BUF>
__device__ __forceinline__ void liquid_cell(const Dev& d, int64_t c, bool valid) {
  using St = Store<S, Q>;
  using T = typename St::T;
  using R = typename St::R;
  const uint8_t fl = valid ? d.flags[c] : (uint8_t)T_GAS;
  const bool mine = (fl & (T_MASK | F_COMPLEX)) == T_LIQ;
  const bool wall = mine && (fl & F_BORDER);
  const bool any_wall = __ballot(wall) != 0ull;
  if (!mine) return;
  const T* A = static_cast<const T*>(d.fA);
  T* B = static_cast<T*>(d.fB);
  const Geom& g = d.g;
  const int64_t stride = g.stride;
  const int64_t nx = g.nx, nxy = (int64_t)g.nx * g.ny;
  R f[Q];
  if (any_wall) {
    // some lane of the wave sits on a no-slip face: per-lane source offsets
    int x, y, z;
    coords(g, c, x, y, z);
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      const int64_t off = kCX[k] + kCY[k] * nx + kCZ[k] * nxy;
      const bool in = (unsigned)(x - kCX[k]) < (unsigned)g.nx &&
                      (unsigned)(y - kCY[k]) < (unsigned)g.ny &&
                      (unsigned)(z - kCZ[k]) < (unsigned)g.nz;
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
      const int64_t off = kCX[k] + kCY[k] * nx + kCZ[k] * nxy;
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

// ---------------------------------------------------------------------------
// List-driven kernels work on one cell per group of 32 lanes: lane k handles
// lattice direction k (lanes >= q idle in the direction work). Sums over
// directions are butterfly reductions over the group: every lane performs the
// same additions (a + b and b + a round alike), so all lanes hold the same,
// deterministic result. The order differs from a sequential loop only by
// rounding.
// ---------------------------------------------------------------------------
constexpr int kG = 32;

// sum over the lanes k < n of the group (callers pass 0 from lanes >= n)
template <typename T>
__device__ __forceinline__ T gsum(T v, int) {
#pragma unroll
  for (int o = kG / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kG);
  return v;
}

// ballot restricted to the calling lane's group (bit k = lane k of the group)
__device__ __forceinline__ uint32_t gballot(bool p) {
  return (uint32_t)(__ballot(p) >> (threadIdx.x & 32));
}

// Collision of one cell held one direction per lane (f = population of this
// lane's direction k); same arithmetic as collide().
template <typename R, int Q, bool TRT, bool SH>
__device__ __forceinline__ R gcollide(R f, int k, const CollideParams<R>& cp, R& rho, R& ux, R& uy,
                                      R& uz) {
  const bool act = k < Q;
  const int kk = act ? k : 0;
  const int cx = kCX[kk], cy = kCY[kk], cz = kCZ[kk];
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

// Interface cells (free-surface condition, mass exchange, fill level, mark)
// and liquid cells next to walls or obstacles (streaming with walls only).
template <int S, int Q, bool TRT>
__global__ __launch_bounds__(kBlock) void k_generic(Dev d) {
  using St = Store<S, Q>;
  using T = typename St::T;
  using R = typename St::R;
  constexpr bool SH = St::kShift;
  const T* A = static_cast<const T*>(d.fA);
  T* B = static_cast<T*>(d.fB);
  const Geom& g = d.g;
  const int64_t stride = g.stride;
  const int nif = d.cnt[CNT_IF];
  const int total = nif;
  const int l = threadIdx.x & (kG - 1);
  const bool act = l < Q;
  const int k = act ? l : 0;
  const int kb = opp(k);
  const int cx = kCX[k], cy = kCY[k], cz = kCZ[k];
  const int ngroups = gridDim.x * (kBlock / kG);
  CollideParams<R> cp{R(d.omega), R(d.omega_m), R(d.gx), R(d.gy), R(d.gz), R(d.tau0), R(d.lambda), R(d.cs)};
  for (int item = blockIdx.x * (kBlock / kG) + threadIdx.x / kG; item < total; item += ngroups) {
    const bool is_if = true;
    const int64_t c = d.if_list[item];
    int x, y, z;
    coords(g, c, x, y, z);
    // own post-collision population of this direction and of its opposite
    const R fo = act ? St::ld(A, k * stride + c, k) : R(0);
    const R fo_b = __shfl(fo, kb, kG);
    int64_t src;
    int dir;
    bool wall;
    const int kind = resolve_source<Q>(g, d.flags, x, y, z, k, &src, &dir, &wall);
    R in_val = R(0);
    if (act && kind == SRC_FLUID) in_val = St::ld(A, dir * stride + src, dir);
    R f;
    if (!is_if) {
      if (act && kind == SRC_GAS) atomicOr(&d.cnt[CNT_ERR], ERR_LAYER);
      f = (kind == SRC_FLUID) ? in_val : fo_b;
    } else {
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
      const int v = d.variant;
      const bool nb_based = (v == 1 || v == 2 || (v == 4 && missing < 3));
      bool in_R = ((gas >> k) & 1u) != 0;
      const double phi_c = d.phiA[c];
      if (nb_based) {
        // Parker-Youngs normal (Sec. 2.2): lane l holds phi at offset
        // (l%3-1, (l/3)%3-1, l/9-1); obstacle points take the centre value
        double vphi = phi_c;
        if (l < 27) {
          int64_t j;
          const int t = nb_type(g, d.flags, x, y, z, l % 3 - 1, (l / 3) % 3 - 1, l / 9 - 1, &j);
          vphi = is_obst(t) ? phi_c : d.phiA[j];
        }
        // lane stride of each axis in the 3x3x3 numbering
        double n[3];
#pragma unroll 1
        for (int a = 0; a < 3; ++a) {
          const int sa = a == 0 ? 1 : (a == 1 ? 3 : 9);
          const int s1 = a == 0 ? 3 : (a == 1 ? 9 : 1);
          const int s2 = a == 0 ? 9 : (a == 1 ? 1 : 3);
          double sacc = 0.0;
#pragma unroll 1
          for (int b = -1; b <= 1; ++b) {
            const double wb = b == 0 ? 2.0 : 1.0;
#pragma unroll
            for (int cc = -1; cc <= 1; ++cc) {
              const int lc = 13 + b * s1 + cc * s2;
              const double vp = __shfl(vphi, lc + sa, kG), vm = __shfl(vphi, lc - sa, kG);
              sacc += wb * (cc == 0 ? 2.0 : 1.0) * (vp - vm);
            }
          }
          n[a] = sacc;
        }
        double nmax = fabs(n[0]);
        nmax = fabs(n[1]) > nmax ? fabs(n[1]) : nmax;
        nmax = fabs(n[2]) > nmax ? fabs(n[2]) : nmax;
        const double dot = n[0] * cx + n[1] * cy + n[2] * cz;
        if ((k > 0 || v == 1) && dot >= -d.delta * nmax) in_R = true;
      }
      const R rhoG = d.rhoG ? R(d.rhoG[c]) : R(d.pV[0] * 3.0);
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
        if ((d.flags[src] & T_MASK) == T_LIQ) {
          term = in - out;
        } else {
          const double T_ = d.thurey ? flux_term(d.cls[c], d.cls[src], in, out) : in - out;
          term = 0.5 * (phi_c + d.phiA[src]) * T_;
        }
      }
      const double dm = gsum(term, Q);
      const double rho_n = (SH ? 1.0 : 0.0) + gsum(act ? (double)f : 0.0, Q);
      const double m_new = d.m[c] + dm;
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
        if (mk) atomicAdd(&d.cnt[CNT_MARK0 + (d.step & 1)], 1);
        if (!(m_new == m_new)) atomicOr(&d.cnt[CNT_ERR], ERR_UNSTABLE);
      }
      if (mk && l < 27) {
        // the conversion pass re-types the 3x3x3 neighbourhood of a marked
        // cell (every writer stores the same value)
        int w;
        const int64_t j = nb_index(g, x, y, z, l % 3 - 1, (l / 3) % 3 - 1, l / 9 - 1, &w);
        if (j >= 0) {
          d.cand[j] = 1;
          d.tile_dirty[j / kConvTile] = 1;
        }
      }
    }
    R rho, vx, vy, vz;
    const R fs = gcollide<R, Q, TRT, SH>(f, l, cp, rho, vx, vy, vz);
    if (l == 0 && unstable(rho, vx, vy, vz)) atomicOr(&d.cnt[CNT_ERR], ERR_UNSTABLE);
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
  R f[Q];
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
    f[k] = St::ld(A, dir * stride + src, dir);
  }
  CollideParams<R> cp{R(d.omega), R(d.omega_m), R(d.gx), R(d.gy), R(d.gz), R(d.tau0), R(d.lambda), R(d.cs)};
  R rho, ux, uy, uz;
  collide_any<R, Q, TRT, St::kShift>(f, cp, rho, ux, uy, uz);
  if (unstable(rho, ux, uy, uz)) atomicOr(&d.cnt[CNT_ERR], ERR_UNSTABLE);
#pragma unroll
  for (int k = 0; k < Q; ++k) St::st(B, k * stride + c, k, f[k]);
}

template <int S, int Q, bool TRT>
__global__ __launch_bounds__(kBlock) void k_border(Dev d) {
  const int n = d.cnt[CNT_GEN];
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
    border_cell<S, Q, TRT>(d, d.gen_list[i]);
}

// Each wave takes 64-cell chunks from the chunk list (chunks without liquid
// cells are never visited), one cell per lane.
template <int S, int Q, bool TRT, bool BUF>
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
    liquid_cell<S, Q, TRT, BUF>(d, c, c < d.g.N);
  }
}

// ---------------------------------------------------------------------------
// k_convert: new types from marks, in place, plus compaction.
// ---------------------------------------------------------------------------
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

// Marks of the q-1 stencil neighbours of c, gathered with independent loads;
// returns a bit set: bit 0 some neighbour is marked to-liquid, bit 1 some
// neighbour is marked to-gas. (Only interface cells carry marks.)
template <int Q>
__device__ __forceinline__ int nb_marks(const Dev& d, int64_t c, bool border) {
  const Geom& g = d.g;
  int x = 0, y = 0, z = 0;
  if (border) coords(g, c, x, y, z);
  const int64_t nx = g.nx, nxy = (int64_t)g.nx * g.ny;
  int acc = 0;
#pragma unroll
  for (int k = 1; k < Q; ++k) {
    int64_t j;
    if (!border) {
      j = c + kCX[k] + kCY[k] * nx + kCZ[k] * nxy;
    } else {
      int w;
      j = nb_index(g, x, y, z, kCX[k], kCY[k], kCZ[k], &w);
    }
    const uint8_t m = j >= 0 ? d.mark[j] : (uint8_t)MK_NONE;
    acc |= m;  // MK_L = 1, MK_G = 2
  }
  return acc;
}

// New cell type of cell c from its flags and the marks around it.
template <int Q>
__device__ __forceinline__ uint8_t new_flags(const Dev& d, int64_t c, uint8_t fl) {
  const Geom& g = d.g;
  const int t = fl & T_MASK;
  int nt = t;
  uint8_t bits = 0;
  const bool border = (fl & F_BORDER) != 0;
  const uint8_t mk = (t == T_IF) ? d.mark[c] : (uint8_t)MK_NONE;
  if (t == T_GAS || t == T_LIQ || (t == T_IF && mk != MK_NONE)) {
    const int around = nb_marks<Q>(d, c, border);
    if (t == T_IF) {
      // a to-gas mark next to a to-liquid mark is dropped (Sec. 2.2:
      // separation of liquid and gas has priority)
      if (mk == MK_L) {
        nt = T_LIQ;
        bits = F_CONV;
      } else if (!(around & MK_L)) {
        nt = T_GAS;
        bits = F_CONV;
      }
    } else if (t == T_GAS) {
      if (around & MK_L) {
        nt = T_IF;
        bits = F_NEW_GAS;
      }
    } else if (around & MK_G) {
      // liquid next to a to-gas mark: becomes interface if that mark survives
      int x = 0, y = 0, z = 0;
      if (border) coords(g, c, x, y, z);
      const int64_t nx = g.nx, nxy = (int64_t)g.nx * g.ny;
#pragma unroll 1
      for (int k = 1; k < Q; ++k) {
        int64_t j;
        if (!border) {
          j = c + kCX[k] + kCY[k] * nx + kCZ[k] * nxy;
        } else {
          int w;
          j = nb_index(g, x, y, z, kCX[k], kCY[k], kCZ[k], &w);
          if (j < 0) continue;
        }
        if (d.mark[j] == MK_G && !(nb_marks<Q>(d, j, (d.flags[j] & F_BORDER) != 0) & MK_L)) {
          nt = T_IF;
          bits = F_NEW_LIQ;
          break;
        }
      }
    }
  }
  return (uint8_t)((fl & F_STATIC) | nt | bits);
}


// Block-wide exclusive scan of a per-thread count (wave prefix by shuffles,
// wave totals through LDS). Returns the prefix; *total receives the block sum.
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
  for (int w = 0; w < kBlock / 64; ++w) {
    if (w < wv) before += sh[w];
    tot += sh[w];
  }
  __syncthreads();
  *total = tot;
  return before + inc - v;
}

// Conversion pass. A tile is kConvTile = 16384 consecutive cells; thread t
// owns the 64 cells [64t, 64t+64) of the tile (one chunk), read as four
// 16-byte vectors. Only cells flagged as candidates (the 3x3x3 neighbourhood
// of a marked cell) are re-typed; every cell's transient bits of an earlier
// conversion are cleared. The interface list, the converted list, the chunk
// list and the list of COMPLEX liquid cells are then compacted in ascending
// cell order: block scan of the per-thread counts, decoupled look-back over
// the tiles (one wave per list), each thread writing its own entries.
template <int Q>
__global__ __launch_bounds__(kBlock) void k_convert(Dev d, int rebuild_only) {
  if (!rebuild_only && d.cnt[CNT_MARK0 + (d.step & 1)] == 0) return;
  __shared__ int s_tile;
  __shared__ uint32_t s_scan[4][kBlock / 64];
  __shared__ uint32_t s_excl[4];
  if (threadIdx.x == 0) s_tile = atomicAdd(&d.cnt[CNT_TICKET], 1);
  __syncthreads();
  const int tile = s_tile;
  const uint32_t epoch = (uint32_t)d.cnt[CNT_EPOCH];
  const int64_t base = (int64_t)tile * kConvTile + (int64_t)kConvPer * threadIdx.x;
  const bool update = !rebuild_only && d.tile_dirty[tile];
  const int64_t N = d.g.N;
  uint64_t mif = 0, mcv = 0, mgn = 0, mlq = 0;
  // the next 16-byte vectors are requested before the current ones are processed
  auto load16 = [&](int v, uint4& f16, uint4& c16) {
    const int64_t b0 = base + 16 * v;
    f16 = make_uint4(0, 0, 0, 0);
    c16 = make_uint4(0, 0, 0, 0);
    if (v < kConvPer / 16 && b0 + 16 <= N) {
      f16 = *reinterpret_cast<const uint4*>(d.flags + b0);
      if (update) c16 = *reinterpret_cast<const uint4*>(d.cand + b0);
    }
  };
  uint4 nf16, nc16;
  load16(0, nf16, nc16);
#pragma unroll 1
  for (int v = 0; v < kConvPer / 16; ++v) {
    const int64_t b0 = base + 16 * v;
    union V16 {
      uint4 v;
      uint8_t b[16];
    } fl, cand;
    const bool full = b0 + 16 <= N;
    fl.v = nf16;
    cand.v = nc16;
    load16(v + 1, nf16, nc16);
    if (!full) {
      for (int j = 0; j < 16 && b0 + j < N; ++j) {
        fl.b[j] = d.flags[b0 + j];
        if (update) cand.b[j] = d.cand[b0 + j];
      }
    }
    bool changed = false, any_cand = false;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      if (b0 + j >= N) break;
      const uint8_t f0 = fl.b[j];
      uint8_t nf = f0 & (uint8_t)~F_TRANSIENT;
      if (cand.b[j]) {
        any_cand = true;
        nf = new_flags<Q>(d, b0 + j, f0);
      }
      changed |= (nf != f0);
      fl.b[j] = nf;
      const uint64_t bit = 1ull << (16 * v + j);
      if ((nf & T_MASK) == T_IF) mif |= bit;
      if (nf & F_CONV) mcv |= bit;
      if ((nf & (T_MASK | F_COMPLEX)) == (T_LIQ | F_COMPLEX)) mgn |= bit;
      if ((nf & (T_MASK | F_COMPLEX)) == T_LIQ) mlq |= bit;
    }
    if (changed) {
      if (full) {
        *reinterpret_cast<uint4*>(d.flags + b0) = fl.v;
      } else {
        for (int j = 0; j < 16 && b0 + j < N; ++j) d.flags[b0 + j] = fl.b[j];
      }
    }
    if (any_cand) {
      if (full) {
        *reinterpret_cast<uint4*>(d.cand + b0) = make_uint4(0, 0, 0, 0);
      } else {
        for (int j = 0; j < 16 && b0 + j < N; ++j) d.cand[b0 + j] = 0;
      }
    }
  }
  const uint32_t cch = mlq ? 1u : 0u;  // this thread's cells are one chunk
  const uint32_t cnts[4] = {(uint32_t)__popcll(mif), (uint32_t)__popcll(mcv), cch,
                            (uint32_t)__popcll(mgn)};
  uint32_t pre[4], tot[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) pre[i] = block_excl_scan(cnts[i], s_scan[i], &tot[i]);
  if (threadIdx.x == 0 && update) d.tile_dirty[tile] = 0;
  {
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    unsigned long long* st =
        wv == 0 ? d.scan_if : (wv == 1 ? d.scan_cv : (wv == 2 ? d.scan_ch : d.scan_gen));
    const uint32_t e = lookback_wave(st, tile, tot[wv], epoch, &d.cnt[CNT_ERR]);
    if (lane == 0) s_excl[wv] = e;
  }
  __syncthreads();
  uint32_t o0 = s_excl[0] + pre[0], o1 = s_excl[1] + pre[1], o3 = s_excl[3] + pre[3];
  for (uint64_t m = mif; m; m &= m - 1) d.if_list[o0++] = (int32_t)(base + __builtin_ctzll(m));
  for (uint64_t m = mcv; m; m &= m - 1) d.conv_list[o1++] = (int32_t)(base + __builtin_ctzll(m));
  for (uint64_t m = mgn; m; m &= m - 1) d.gen_list[o3++] = (int32_t)(base + __builtin_ctzll(m));
  if (cch) d.chunk_list[s_excl[2] + pre[2]] = (int32_t)(base / 64);
  if (tile == (int)gridDim.x - 1 && threadIdx.x == kBlock - 1) {
    d.cnt[CNT_IF] = (int32_t)o0;
    d.cnt[CNT_CONV] = (int32_t)o1;
    d.cnt[CNT_GEN] = (int32_t)o3;
    d.cnt[CNT_CHUNKS] = (int32_t)(s_excl[2] + pre[2] + cch);
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
#pragma unroll 1
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

// Completion of one interface cell of the new list by a group of 32 lanes,
// lane k looking at the neighbour x + c_k.
template <int S, int Q, bool TRT>
__device__ __forceinline__ void finish_interface(const Dev& d, int64_t c, int l,
                                                 bool classes_only) {
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
  int w;
  int64_t j = -1;
  uint8_t fj = 0;
  if (act && l > 0) {
    j = nb_index(g, x, y, z, kCX[k], kCY[k], kCZ[k], &w);
    if (j >= 0) fj = d.flags[j];
  }
  const int tj = j >= 0 ? (fj & T_MASK) : -1;
  const bool has_liq = gballot(tj == T_LIQ) != 0u;
  const bool has_gas = gballot(tj == T_GAS) != 0u;
  const uint8_t cls = (!has_liq && has_gas) ? CLS_NOLIQ : ((!has_gas && has_liq) ? CLS_NOGAS : CLS_STD);
  if (classes_only) {
    if (l == 0) d.cls[c] = cls;
    return;
  }
  const uint8_t fl = d.flags[c];
  double mass, rho_n;
  if (fl & F_NEW_GAS) {
    // equilibrium of the mean density and velocity of the liquid and old
    // interface neighbours (Sec. 2.2), then the collision of this step
    const bool use = j >= 0 && is_fluid(tj) && !(fj & F_NEW_GAS);
    R r = R(0), a = R(0), b = R(0), cc = R(0);
    if (use) {
      R fj_[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) fj_[i] = St::ld(B, i * stride + j, i);
      post_moments<R, Q, SH>(fj_, R(d.gx), R(d.gy), R(d.gz), r, a, b, cc);
    }
    const int cnt = __popc(gballot(use));
    const R rb = gsum(r, Q) / R(cnt);
    const R ub0 = gsum(a, Q) / R(cnt), ub1 = gsum(b, Q) / R(cnt), ub2 = gsum(cc, Q) / R(cnt);
    const R usq = ub0 * ub0 + ub1 * ub1 + ub2 * ub2;
    const R fe = feq_k<R, Q, SH>(k, rb, rb - R(1), cdot<R>(kCX[k], kCY[k], kCZ[k], ub0, ub1, ub2),
                                 usq);
    CollideParams<R> cp{R(d.omega), R(d.omega_m), R(d.gx), R(d.gy), R(d.gz), R(d.tau0), R(d.lambda), R(d.cs)};
    R rr, vx, vy, vz;
    const R fs = gcollide<R, Q, TRT, SH>(fe, l, cp, rr, vx, vy, vz);
    if (act) St::st(B, k * stride + c, k, fs);
    mass = 0.0;
    rho_n = (double)rb;
  } else if (fl & F_NEW_LIQ) {
    const R fc = act ? St::ld(B, k * stride + c, k) : R(0);
    rho_n = (SH ? 1.0 : 0.0) + gsum(act ? (double)fc : 0.0, Q);
    mass = rho_n;
  } else {
    mass = d.m[c];
    rho_n = d.rho_if[c];
  }
  // excess mass of converted neighbours: equal shares over their interface
  // neighbours (Sec. 2.2), added in direction order
  double share = 0.0;
  if (j >= 0 && (fj & F_CONV)) share = excess_of(d, j) / (double)count_if_nb<Q>(d, j);
  for (int i = 1; i < Q; ++i) {
    const double si = __shfl(share, i, kG);
    if (__shfl((int)((fj & F_CONV) != 0), i, kG)) mass += si;
  }
  if (l == 0) {
    d.m[c] = mass;
    d.rho_if[c] = rho_n;
    d.phiB[c] = mass / rho_n;
    d.cls[c] = cls;
  }
}

template <int Q>
__device__ __forceinline__ void finish_converted(const Dev& d, int64_t z, int l) {
  const bool act = l < Q;
  int x, y, zz;
  coords(d.g, z, x, y, zz);
  bool nbif = false;
  if (act && l > 0) {
    int w;
    const int64_t j = nb_index(d.g, x, y, zz, kCX[l], kCY[l], kCZ[l], &w);
    nbif = j >= 0 && (d.flags[j] & T_MASK) == T_IF;
  }
  const int nif = __popc(gballot(nbif));
  if (l == 0) {
    const int t = d.flags[z] & T_MASK;
    if (nif == 0) d.lost[z] += excess_of(d, z);
    d.mark[z] = MK_NONE;
    const double v = (t == T_LIQ) ? 1.0 : 0.0;
    d.phiA[z] = v;
    d.phiB[z] = v;
  }
}

template <int S, int Q, bool TRT>
__global__ __launch_bounds__(kBlock) void k_finish(Dev d, int classes_only) {
  if (!classes_only && d.cnt[CNT_MARK0 + (d.step & 1)] == 0) return;
  const int nif = d.cnt[CNT_IF];
  const int ncv = classes_only ? 0 : d.cnt[CNT_CONV];
  const int total = nif + ncv;
  const int l = threadIdx.x & (kG - 1);
  const int ngroups = gridDim.x * (kBlock / kG);
  for (int item = blockIdx.x * (kBlock / kG) + threadIdx.x / kG; item < total; item += ngroups) {
    if (item < nif)
      finish_interface<S, Q, TRT>(d, d.if_list[item], l, classes_only != 0);
    else
      finish_converted<Q>(d, d.conv_list[item - nif], l);
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
  bool complex_ = false;
  bool gas_nb = false;
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int r[3] = {x + dx, y + dy, z + dz};
        const int n[3] = {g.nx, g.ny, g.nz};
        for (int a = 0; a < 3; ++a) {
          const int face = r[a] < 0 ? 2 * a : (r[a] >= n[a] ? 2 * a + 1 : -1);
          if (face >= 0 && g.bnd[face] != BND_NOSLIP) complex_ = true;
        }
        int w;
        int64_t j = nb_index(g, x, y, z, dx, dy, dz, &w);
        if (j < 0) continue;
        const int tj = d.flags[j] & T_MASK;
        if (is_obst(tj)) border = complex_ = true;
      }
  for (int k = 1; k < Q; ++k) {
    int w;
    int64_t j = nb_index(g, x, y, z, kCX[k], kCY[k], kCZ[k], &w);
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
