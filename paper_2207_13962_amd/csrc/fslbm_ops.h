// Context, device memory layout and the per-format kernel table of libfslbm.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "fslbm.h"
#include <hip/hip_ext.h>
#include "fslbm_kernels.h"
#include "fslbm_batch.h"

using namespace fslbm;

namespace fslbm_host {

inline int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

inline int storage_bytes(int storage) { return storage == FSLBM_F64 ? 8 : (storage == FSLBM_F32 ? 4 : 2); }

// Device memory layout (one arena, 256-byte aligned sub-buffers).
struct Layout {
  int64_t N, stride, tiles, conv_per, red_blocks;
  int64_t stash_cap;  // in place: entries of one stash buffer (0: two grids)
  size_t off_stash, off_prevpos;
  size_t off_fA, off_fB, off_flags, off_mark, off_cls, off_phiA, off_phiB, off_m, off_rho_if,
      off_rhoG, off_phis, off_smap, off_lost, off_if_list, off_conv_list, off_chunk_list, off_chunk_mask, off_gen_list,
      off_mark_list, off_ng_list, off_nl_list, off_cnt, off_scan_status,
      off_pv, off_partial, off_stage, off_blab, off_bpar, off_btgt, off_bV, off_bW, off_bR, off_bnn,
      off_bVl, off_bWl, off_bRl, off_bnnl,
      off_bamt, off_bpr, off_bhas, total;
};


inline Layout make_layout(const fslbm_params& p) {
  Layout L{};
  L.N = (int64_t)p.nx * p.ny * p.nz;
  L.stride = round_up(L.N, 256);
  // compaction: cells per thread 16 times a power of two, at most kMaxTiles tiles
  L.conv_per = 16;
  while (L.conv_per * kCompBlock * kMaxTiles < L.N) L.conv_per *= 2;
  L.tiles = (L.N + kCompBlock * L.conv_per - 1) / (kCompBlock * L.conv_per);
  L.red_blocks = (L.N + kRedCells - 1) / kRedCells;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += (size_t)round_up((int64_t)bytes, 256);
    return at;
  };
  const size_t pdf = (size_t)p.q * (size_t)L.stride * storage_bytes(p.storage);
  const bool aa = p.layout == FSLBM_AA;
  L.off_fA = take(pdf);
  L.off_fB = aa ? L.off_fA : take(pdf);
  // in place: two stash buffers of the interface cells' own populations and
  // the per-cell entry index. A buffer holds an eighth of the domain, or twice
  // its largest face for flat domains (a surface spanning that face), at
  // least 1024 cells and at most all.
  const int64_t face = std::max({(int64_t)p.nx * p.ny, (int64_t)p.ny * p.nz, (int64_t)p.nx * p.nz});
  L.stash_cap = aa ? std::min<int64_t>(L.N, std::max({L.N / 8, 2 * face, (int64_t)1024})) : 0;
  L.off_stash = take(2 * (size_t)L.stash_cap * p.q * storage_bytes(p.storage));
  L.off_prevpos = take(aa ? 4 * (size_t)L.N : 0);
  L.off_flags = take(L.N + 16);
  L.off_mark = take(L.N);
  L.off_cls = take(L.N);
  L.off_phiA = take(8 * L.N);
  L.off_phiB = take(8 * L.N);
  L.off_m = take(8 * L.N);
  L.off_rho_if = take(8 * L.N);
  const bool tracked = p.bubble_model == 2;
  L.off_rhoG = take(p.sigma != 0.0 || tracked ? 8 * L.N : 0);
  L.off_phis = take(p.sigma != 0.0 ? 8 * L.N : 0);
  L.off_smap = take(p.sigma != 0.0 ? 4 * (size_t)smooth_tiles(p.nx, p.ny, p.nz) : 0);
  L.off_lost = take(8 * L.N);
  L.off_if_list = take(4 * L.N);
  L.off_conv_list = take(4 * L.N);
  L.off_chunk_list = take(4 * (L.N / 64 + 1));
  L.off_chunk_mask = take(8 * (L.N / 64 + 1));
  L.off_gen_list = take(4 * L.N);
  L.off_mark_list = take(4 * L.N);
  L.off_ng_list = take(4 * L.N);
  L.off_nl_list = take(4 * L.N);
  L.off_cnt = take(4 * CNT_N);
  L.off_scan_status = take(16 * L.tiles);
  L.off_pv = take(8 * 8);
  L.off_partial = take(8 * kRedN * L.red_blocks + 8 * 16);
  // staging of one population plane; at creation also the slot bitmap of
  // the in-place layout (q * stride bits)
  L.off_stage = take(std::max<size_t>(8 * L.N, (size_t)p.q * L.stride / 8 + 8));
  L.off_blab = take(tracked ? 4 * L.N : 0);
  L.off_bpar = take(tracked ? 4 * L.N : 0);
  L.off_btgt = take(tracked ? 4 * L.N : 0);
  L.off_bV = take(tracked ? 8 * L.N : 0);
  L.off_bW = take(tracked ? 8 * L.N : 0);
  L.off_bR = take(tracked ? 8 * L.N : 0);
  L.off_bnn = take(tracked ? 8 * L.N : 0);
  L.off_bVl = take(tracked ? 8 * L.N : 0);
  L.off_bWl = take(tracked ? 8 * L.N : 0);
  L.off_bRl = take(tracked ? 8 * L.N : 0);
  L.off_bnnl = take(tracked ? 8 * L.N : 0);
  L.off_bamt = take(tracked ? 8 * L.N : 0);
  L.off_bpr = take(tracked ? 8 * L.N : 0);
  L.off_bhas = take(tracked ? L.N : 0);
  L.total = o;
  return L;
}

inline const char* validate(const fslbm_params* p) {
  if (!p) return "params is NULL";
  if (p->abi_version != FSLBM_ABI_VERSION) return "abi_version mismatch";
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return "nx, ny, nz must be >= 1";
  if ((int64_t)p->nx * p->ny * p->nz >= (1LL << 30)) return "domain larger than 2^30 cells";
  if (p->q != 19 && p->q != 27) return "q must be 19 or 27";
  if (p->collision != FSLBM_SRT && p->collision != FSLBM_TRT) return "unknown collision operator";
  if (p->storage < FSLBM_F64 || p->storage > FSLBM_F16S) return "unknown storage format";
  for (int f = 0; f < 6; ++f)
    if (p->boundary[f] < FSLBM_PERIODIC || p->boundary[f] > FSLBM_WALL_FREESLIP)
      return "unknown boundary kind";
  for (int a = 0; a < 3; ++a)
    if ((p->boundary[2 * a] == FSLBM_PERIODIC) != (p->boundary[2 * a + 1] == FSLBM_PERIODIC))
      return "a periodic face needs a periodic opposite face";
  if (p->variant < FSLBM_NBRC || p->variant > FSLBM_OM3) return "unknown variant";
  if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return "tau must be > 0.5";
  if (p->collision == FSLBM_TRT && !(p->trt_lambda > 0.0)) return "trt_lambda must be > 0";
  if (!(p->rho_gas > 0.0)) return "rho_gas must be > 0";
  if (!(p->eps_phi >= 0.0)) return "eps_phi must be >= 0";
  if (p->sigma < 0.0) return "sigma must be >= 0";
  if (!(p->smagorinsky >= 0.0)) return "smagorinsky must be >= 0";
  if (p->bubble_model < 0 || p->bubble_model > 2) return "bubble_model must be 0, 1 or 2";
  if (p->layout != FSLBM_TWO_GRID && p->layout != FSLBM_AA) return "unknown layout";
  return nullptr;
}

}  // namespace fslbm_host

struct fslbm_ctx {
  fslbm_params p;
  fslbm_host::Layout L;
  hipStream_t stream = nullptr;
  char* arena = nullptr;
  bool own_arena = false;
  Dev d{};
  int64_t step = 0;
  int status = FSLBM_OK;  // sticky device / runtime failure
  std::string last_error;
  // optional events around the liquid stream-collide launches
  std::vector<hipEvent_t> ev;
  int64_t ev_used = 0;
  // captured launch sequences of kGraphSteps and of 2 steps (even counts, so
  // the grid and fill-level buffers and the counter slots return to where
  // they started), one of each per step parity (the parity decides which
  // buffers and counter slots the captured launches use); replayed while no
  // parameter changes
  hipGraph_t graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};            // [length][parity]
  hipGraphExec_t graph_exec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  bool graphs = true;
  int cus = 256;  // compute units of the device
  int device = 0;  // the device current at creation (the arena's device)
};

constexpr int64_t kGraphSteps = 8;


namespace fslbm_host {

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// interface blocks of k_step: enough to cover a large interface list with few
// launches' worth of work per thread
// persistent-style grid of the liquid kernel: about the waves the GPU holds
// at this kernel's occupancy, capped by the number of chunks
inline unsigned liquid_blocks(const fslbm_ctx* c) {
  const int64_t chunks = c->L.N / 64 + 1;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((chunks + 3) / 4, 256 * 7));
}

inline unsigned border_blocks(const fslbm_ctx* c) {
  int64_t b = grid_for(c->L.N) / 16 + 64;
  return (unsigned)std::min<int64_t>(b, 2048);
}

// list kernels with one cell per 32-lane group: about one group per list
// entry for typical interface fractions, capped at what 256 CUs hold at the
// kernels' occupancy (four 256-thread blocks per CU)
inline unsigned if_blocks(const fslbm_ctx* c) {
  int64_t b = grid_for(c->L.N) / 8 + 64;
  return (unsigned)std::min<int64_t>(b, 1024);
}

// groups of k_retype: the marks of one step are a small part of the interface
inline unsigned retype_blocks(const fslbm_ctx* c) {
  int64_t b = grid_for(c->L.N) / 64 + 16;
  return (unsigned)std::min<int64_t>(b, 512);
}

// k_curvature: one 32-lane group per interface cell, about two cells per
// group at typical interface fractions
inline unsigned curv_blocks(const fslbm_ctx* c) {
  int64_t b = grid_for(c->L.N) / 8 + 16;
  return (unsigned)std::min<int64_t>(b, 2048);
}

// k_classes: one thread per interface cell
inline unsigned list_blocks(const fslbm_ctx* c) {
  int64_t b = grid_for(c->L.N) / 32 + 16;
  return (unsigned)std::min<int64_t>(b, 512);
}

// worker blocks of the compaction: about one thread per (changed cell,
// direction) pair at typical conversion rates, growing with the domain, but
// fewer where the tiles already take most of the GPU (whole step with 256
// workers beside 128 tiles 2 % faster than with 128 on a 2.1 M-cell domain;
// 128 beside 512 tiles 2 % faster than 256 on an 8.4 M-cell one)
inline int compact_workers(const fslbm_ctx* c) {
  const int64_t room = std::min<int64_t>(256, std::max<int64_t>(128, 512 - c->L.tiles));
  return (int)std::max<int64_t>(8, std::min<int64_t>(grid_for(c->L.N) / 32, room));
}

// One batched step over the resident runs of one (storage, lattice,
// collision, addressing) group: device tables of its launches.
constexpr int kLaunches = 3;  // streaming, re-typing, compaction and completion

// Launches beside the step for the runs that need them: smoothing and
// curvature (surface tension) before the streaming launch, the bubble volume
// and volume pressure (single-bubble model) after the compaction.
// Tracked bubbles: the seven bubble passes after the compaction, over a
// run's cells (AUX_BUB) or its wave stretches (AUX_BUBW).
constexpr int kAux = 6;
enum { AUX_SMOOTH = 0, AUX_CURV = 1, AUX_VOL = 2, AUX_SUMVOL = 3, AUX_BUB = 4, AUX_BUBW = 5 };
constexpr int kTabs = kLaunches + kAux;  // tables per group

struct BatchLaunch {
  const Dev* devs = nullptr;
  const BatchEntry* tab[kLaunches] = {nullptr, nullptr, nullptr};  // one table per launch
  int n = 0;                                 // entries of each table (one per run)
  int blocks[kLaunches] = {0, 0, 0};         // blocks of each launch
  bool buf = true;                 // buffer addressing (every grid below 2 GiB)
  bool aa = false;                 // in-place layout
  int q = 19;                      // lattice of the group
  const BatchEntry* aux[kAux] = {};  // only the runs that need them
  int aux_n[kAux] = {};
  int aux_blocks[kAux] = {};
};

// Kernel table for one (storage, lattice, collision) combination.
struct Ops {
  void (*step)(fslbm_ctx*, hipStream_t);
  void (*convert)(fslbm_ctx*, hipStream_t, int rebuild_only);
  void (*classes)(fslbm_ctx*, hipStream_t);
  void (*reduce_mass)(const Dev&, int64_t blocks, hipStream_t);  // partials to d.partial
  void (*batch_step)(const BatchLaunch&, hipStream_t, int64_t tick);
  void (*init_state)(fslbm_ctx*, hipStream_t, int resume);
  void (*init_flags)(fslbm_ctx*, hipStream_t);
  void (*import_plane)(fslbm_ctx*, hipStream_t, const double*, int);
  void (*export_field)(fslbm_ctx*, hipStream_t, double*, int);
  void (*aa_check)(fslbm_ctx*, hipStream_t, uint32_t*);
  void (*stash_init)(fslbm_ctx*, hipStream_t);
};

template <int S, int Q, bool TRT>
struct Impl {
  static void step(fslbm_ctx* c, hipStream_t s) {
    // buffer addressing when a population grid spans less than 2 GiB
    const bool buf = (double)Q * (double)c->L.stride * sizeof(typename Store<S, Q>::T) < 2147483648.0;
    // with timing on, the streaming kernel's own dispatch records start/stop
    // timestamps (no separate event packets around it)
    const bool timed = 2 * (c->ev_used + 1) <= (int64_t)c->ev.size();
    hipEvent_t e0 = timed ? c->ev[2 * c->ev_used] : nullptr;
    hipEvent_t e1 = timed ? c->ev[2 * c->ev_used + 1] : nullptr;
    if (timed) c->ev_used++;
    // role split of the streaming launch, in units of what the GPU holds at
    // once (four 256-thread blocks per CU at the kernel's occupancy): 3/8 for
    // the interface groups, 1/8 for the wall-liquid cells, 5/8 for the liquid
    // chunks (the liquid blocks beyond the first wave fill the CUs that the
    // short-lived roles leave; measured on dam256: 22.2 us per launch against
    // 23.7 us with 1/2)
    // (role sizes are multiples of the XCD count, so that a role's block index
    // modulo kXcds is the XCD the block runs on)
    const int64_t cap = 4 * (int64_t)c->cus;
    auto xr = [](int64_t b) { return (int)std::max<int64_t>(kXcds, (b + kXcds - 1) / kXcds * kXcds); };
    const int gen = xr(std::min<int64_t>(if_blocks(c), cap * 3 / 8));
    const int bord = xr(std::min<int64_t>(border_blocks(c), cap / 8));
    const int liq = xr(std::min<int64_t>(liquid_blocks(c), cap * 5 / 8));
    const dim3 grid((unsigned)(gen + bord + liq));
    if (c->d.aa) {
      if (buf)
        hipExtLaunchKernelGGL((k_stream<S, Q, TRT, true, true>), grid, dim3(kBlock), 0, s, e0, e1, 0, c->d,
                              gen, bord);
      else
        hipExtLaunchKernelGGL((k_stream<S, Q, TRT, false, true>), grid, dim3(kBlock), 0, s, e0, e1, 0, c->d,
                              gen, bord);
    } else if (buf) {
      hipExtLaunchKernelGGL((k_stream<S, Q, TRT, true, false>), grid, dim3(kBlock), 0, s, e0, e1, 0, c->d,
                            gen, bord);
    } else {
      hipExtLaunchKernelGGL((k_stream<S, Q, TRT, false, false>), grid, dim3(kBlock), 0, s, e0, e1, 0, c->d,
                            gen, bord);
    }
  }
  static void convert(fslbm_ctx* c, hipStream_t s, int rebuild) {
    hipLaunchKernelGGL((k_retype<Q>), dim3(retype_blocks(c)), dim3(kBlock), 0, s, c->d, rebuild);
    const int workers = rebuild ? 0 : compact_workers(c);
    if (c->d.aa)
      hipLaunchKernelGGL((k_compact<S, Q, TRT, true>), dim3((unsigned)(c->L.tiles + workers)),
                         dim3(kCompBlock), 0, s, c->d, rebuild, (int)c->L.conv_per, workers);
    else
      hipLaunchKernelGGL((k_compact2<S, Q, TRT>), dim3((unsigned)(c->L.tiles + workers)),
                         dim3(kCompBlock), 0, s, c->d, (int)c->L.conv_per, rebuild ? -1 : workers);
  }
  static void classes(fslbm_ctx* c, hipStream_t s) {
    hipLaunchKernelGGL((k_classes<Q>), dim3(list_blocks(c)), dim3(kBlock), 0, s, c->d);
  }
  static void batch_step(const BatchLaunch& bl, hipStream_t s, int64_t tick) {
    if (bl.n == 0) return;
    if (bl.aa) {
      if (bl.buf)
        hipLaunchKernelGGL((kb_stream<S, Q, TRT, true, true>), dim3((unsigned)bl.blocks[0]), dim3(kBlock), 0,
                           s, bl.devs, bl.tab[0], bl.n, tick);
      else
        hipLaunchKernelGGL((kb_stream<S, Q, TRT, false, true>), dim3((unsigned)bl.blocks[0]), dim3(kBlock), 0,
                           s, bl.devs, bl.tab[0], bl.n, tick);
    } else if (bl.buf) {
      hipLaunchKernelGGL((kb_stream<S, Q, TRT, true, false>), dim3((unsigned)bl.blocks[0]), dim3(kBlock), 0, s,
                         bl.devs, bl.tab[0], bl.n, tick);
    } else {
      hipLaunchKernelGGL((kb_stream<S, Q, TRT, false, false>), dim3((unsigned)bl.blocks[0]), dim3(kBlock), 0, s,
                         bl.devs, bl.tab[0], bl.n, tick);
    }
    hipLaunchKernelGGL((kb_retype<Q>), dim3((unsigned)bl.blocks[1]), dim3(kBlock), 0, s, bl.devs, bl.tab[1],
                       bl.n, tick);
    if (bl.aa)
      hipLaunchKernelGGL((kb_compact<S, Q, TRT, true>), dim3((unsigned)bl.blocks[2]), dim3(kCompBlock), 0, s,
                         bl.devs, bl.tab[2], bl.n, tick);
    else
      hipLaunchKernelGGL((kb_compact<S, Q, TRT, false>), dim3((unsigned)bl.blocks[2]), dim3(kCompBlock), 0, s,
                         bl.devs, bl.tab[2], bl.n, tick);
  }
  static void reduce_mass(const Dev& d, int64_t blocks, hipStream_t s) {
    hipLaunchKernelGGL((k_reduce_mass<S, Q>), dim3((unsigned)blocks), dim3(kBlock), 0, s, d, kRedCells);
  }
  static void init_state(fslbm_ctx* c, hipStream_t s, int resume) {
    hipLaunchKernelGGL((k_init_state<S, Q, TRT>), dim3(grid_for(c->L.N)), dim3(kBlock), 0, s, c->d,
                       resume);
  }
  static void init_flags(fslbm_ctx* c, hipStream_t s) {
    hipLaunchKernelGGL((k_init_flags<Q>), dim3(grid_for(c->L.N)), dim3(kBlock), 0, s, c->d);
  }
  static void import_plane(fslbm_ctx* c, hipStream_t s, const double* src, int k) {
    hipLaunchKernelGGL((k_import_plane<S, Q>), dim3(grid_for(c->L.N)), dim3(kBlock), 0, s, c->d,
                       src, k);
  }
  static void export_field(fslbm_ctx* c, hipStream_t s, double* out, int what) {
    hipLaunchKernelGGL((k_export<S, Q>), dim3(grid_for(c->L.N)), dim3(kBlock), 0, s, c->d, out,
                       what);
  }
  static void aa_check(fslbm_ctx* c, hipStream_t s, uint32_t* bits) {
    hipLaunchKernelGGL((k_aa_check<Q>), dim3(grid_for(c->L.N)), dim3(kBlock), 0, s, c->d, bits);
  }
  static void stash_init(fslbm_ctx* c, hipStream_t s) {
    hipLaunchKernelGGL((k_stash_init<S, Q>), dim3(if_blocks(c)), dim3(kBlock), 0, s, c->d);
  }
  static constexpr Ops ops() {
    return Ops{&step, &convert, &classes, &reduce_mass, &batch_step, &init_state, &init_flags, &import_plane,
               &export_field, &aa_check, &stash_init};
  }
};


Ops ops_f64_q19(int coll);
Ops ops_f64_q27(int coll);
Ops ops_f32_q19(int coll);
Ops ops_f32_q27(int coll);
Ops ops_f16s_q19(int coll);
Ops ops_f16s_q27(int coll);

}  // namespace fslbm_host
