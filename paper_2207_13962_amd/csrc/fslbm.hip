// Host side of libfslbm: context, device memory layout, launches, C ABI.
// The public interface is declared (and documented) in include/fslbm.h.
// The kernels that do not depend on the population format live in this unit.
#define FSLBM_HOST_KERNELS 1
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "fslbm.h"
#include "fslbm_kernels.h"

using namespace fslbm;

#include "fslbm_ops.h"

using namespace fslbm_host;

#include <mutex>

namespace {

thread_local char g_create_error[512] = "";

// Scratch of fslbm_mass_noalloc: the per-block partial sums of the mass
// reduction (kRedN doubles for each block of kRedCells cells), for domains of
// at most kNoAllocBlocks * kRedCells cells. Each GPU the library runs on holds
// its own copy until the process ends. In host code `scratch` is only a
// symbol: its device address on a GPU comes from hipGetSymbolAddress with
// that GPU current (kept in g_scratch, filled by fslbm_create).
constexpr int64_t kNoAllocBlocks = 16384;
__device__ __align__(256) double scratch[kNoAllocBlocks * kRedN];
constexpr int kMaxDevices = 64;
double* g_scratch[kMaxDevices] = {nullptr};
std::mutex g_scratch_mu;

// Address of the scratch array on the current device (resolved once per
// device); nullptr on failure.
double* scratch_for_current_device(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch[dev] = static_cast<double*>(ptr);
  }
  return g_scratch[dev];
}

int set_err(fslbm_ctx* c, int st, const std::string& msg) {
  if (c) c->last_error = msg;
  return st;
}

int hip_fail(fslbm_ctx* c, hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  if (c) {
    c->status = FSLBM_EDEVICE;
    c->last_error = m;
  } else {
    snprintf(g_create_error, sizeof g_create_error, "%s", m.c_str());
  }
  return FSLBM_EDEVICE;
}

#define HIPCHK(ctx, expr)                              \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr); \
  } while (0)

Ops pick(const fslbm_params& p) {
  if (p.storage == FSLBM_F32) return p.q == 27 ? ops_f32_q27(p.collision) : ops_f32_q19(p.collision);
  if (p.storage == FSLBM_F16S) return p.q == 27 ? ops_f16s_q27(p.collision) : ops_f16s_q19(p.collision);
  return p.q == 27 ? ops_f64_q27(p.collision) : ops_f64_q19(p.collision);
}

// The Dev record is every kernel's argument, and its size shows in the
// streaming launch of the 2.1 M-cell dam break: 20.4 us per launch at 504
// bytes, 20.6 at 512, 21.3 at 520 (it holds only what kernels read), so a
// new field must displace another.
static_assert(sizeof(Dev) <= 504, "the kernel-argument record grew past 504 bytes");

void bind(fslbm_ctx* c) {
  const Layout& L = c->L;
  char* a = c->arena;
  Dev& d = c->d;
  d.g.nx = c->p.nx;
  d.g.ny = c->p.ny;
  d.g.nz = c->p.nz;
  d.g.bnd_bits = 0;
  for (int f = 0; f < 6; ++f) {
    d.g.bnd[f] = c->p.boundary[f];
    d.g.bnd_bits |= (uint32_t)c->p.boundary[f] << (2 * f);
  }
  d.g.N = L.N;
  d.g.stride = L.stride;
  const double tau = c->p.tau;
  d.omega = 1.0 / tau;
  d.omega_m = c->p.collision == FSLBM_TRT ? 1.0 / (0.5 + c->p.trt_lambda / (tau - 0.5)) : d.omega;
  d.tau0 = tau;
  d.lambda = c->p.trt_lambda;
  d.cs = c->p.smagorinsky;
  d.gx = c->p.gravity[0];
  d.gy = c->p.gravity[1];
  d.gz = c->p.gravity[2];
  d.sigma = c->p.sigma;
  d.eps = c->p.eps_phi;
  d.delta = c->p.tie_delta > 0.0 ? c->p.tie_delta : 1e-9;
  d.variant = c->p.variant;
  d.thurey = c->p.thurey_flux;
  d.bubble = c->p.bubble_model;
  d.fA = a + L.off_fA;
  d.fB = a + L.off_fB;  // the same grid in place
  d.aa = c->p.layout == FSLBM_AA ? 1 : 0;
  d.stash_cap = (int32_t)L.stash_cap;
  d.stash = d.aa ? a + L.off_stash : nullptr;
  d.prevpos = d.aa ? reinterpret_cast<int32_t*>(a + L.off_prevpos) : nullptr;
  d.flags = reinterpret_cast<uint8_t*>(a + L.off_flags);
  d.mark = reinterpret_cast<uint8_t*>(a + L.off_mark);
  d.cls = reinterpret_cast<uint8_t*>(a + L.off_cls);
  d.phiA = reinterpret_cast<double*>(a + L.off_phiA);
  d.phiB = reinterpret_cast<double*>(a + L.off_phiB);
  d.m = reinterpret_cast<double*>(a + L.off_m);
  d.rho_if = reinterpret_cast<double*>(a + L.off_rho_if);
  const bool tracked = c->p.bubble_model == 2;
  d.rhoG = c->p.sigma != 0.0 || tracked ? reinterpret_cast<double*>(a + L.off_rhoG) : nullptr;
  d.phis = c->p.sigma != 0.0 ? reinterpret_cast<double*>(a + L.off_phis) : nullptr;
  d.smap = c->p.sigma != 0.0 ? reinterpret_cast<int32_t*>(a + L.off_smap) : nullptr;
  d.lost = reinterpret_cast<double*>(a + L.off_lost);
  d.if_list = reinterpret_cast<int32_t*>(a + L.off_if_list);
  d.conv_list = reinterpret_cast<int32_t*>(a + L.off_conv_list);
  d.chunk_list = reinterpret_cast<int32_t*>(a + L.off_chunk_list);
  d.chunk_mask = reinterpret_cast<uint64_t*>(a + L.off_chunk_mask);
  d.gen_list = reinterpret_cast<int32_t*>(a + L.off_gen_list);
  d.mark_list = reinterpret_cast<int32_t*>(a + L.off_mark_list);
  d.ng_list = reinterpret_cast<int32_t*>(a + L.off_ng_list);
  d.nl_list = reinterpret_cast<int32_t*>(a + L.off_nl_list);
  d.cnt = reinterpret_cast<int32_t*>(a + L.off_cnt);
  d.scan_status = reinterpret_cast<unsigned long long*>(a + L.off_scan_status);
  d.pV = reinterpret_cast<double*>(a + L.off_pv);
  d.partial = reinterpret_cast<double*>(a + L.off_partial);
  d.blab = tracked ? reinterpret_cast<int32_t*>(a + L.off_blab) : nullptr;
  d.bpar = tracked ? reinterpret_cast<int32_t*>(a + L.off_bpar) : nullptr;
  d.btgt = tracked ? reinterpret_cast<int32_t*>(a + L.off_btgt) : nullptr;
  d.bV = tracked ? reinterpret_cast<int64_t*>(a + L.off_bV) : nullptr;
  d.bW = tracked ? reinterpret_cast<int64_t*>(a + L.off_bW) : nullptr;
  d.bR = tracked ? reinterpret_cast<int64_t*>(a + L.off_bR) : nullptr;
  d.bnn = tracked ? reinterpret_cast<int64_t*>(a + L.off_bnn) : nullptr;
  d.bVl = tracked ? reinterpret_cast<uint64_t*>(a + L.off_bVl) : nullptr;
  d.bWl = tracked ? reinterpret_cast<uint64_t*>(a + L.off_bWl) : nullptr;
  d.bRl = tracked ? reinterpret_cast<uint64_t*>(a + L.off_bRl) : nullptr;
  d.bnnl = tracked ? reinterpret_cast<uint64_t*>(a + L.off_bnnl) : nullptr;
  d.bamt = tracked ? reinterpret_cast<double*>(a + L.off_bamt) : nullptr;
  d.bpr = tracked ? reinterpret_cast<double*>(a + L.off_bpr) : nullptr;
  d.bhas = tracked ? reinterpret_cast<uint8_t*>(a + L.off_bhas) : nullptr;
}

double* stage(fslbm_ctx* c) { return reinterpret_cast<double*>(c->arena + c->L.off_stage); }

// Bubble volume at t+1 (phiB, new types) and the volume pressure update.
void launch_volume(fslbm_ctx* c, hipStream_t s, bool set_reference) {
  const int64_t blocks = vol_blocks_of(c->L.N);
  hipLaunchKernelGGL(k_reduce_volume, dim3((unsigned)blocks), dim3(kBlock), 0, s, c->d, kVolCells);
  double* out = c->d.partial + kRedN * c->L.red_blocks;
  // with set_reference: p^V(0) = rho_gas / 3 was set by the caller; V(0) = V
  hipLaunchKernelGGL(k_sum_volume, dim3(1), dim3(kBlock), 0, s, c->d.partial, (int)blocks, out, c->d.pV,
                     set_reference ? 1 : 0);
}

// Tracked bubbles from the types and fill levels at t+1 (flags, phiB): new
// labels, volumes, amounts handed over, pressures, gas densities. The
// labelling passes skip a step without marks unless `force` (creation).
void launch_bubbles(fslbm_ctx* c, hipStream_t s, bool force) {
  const dim3 grid(grid_for(c->L.N)), block(kBlock);
  hipLaunchKernelGGL(k_bub_init, grid, block, 0, s, c->d, force ? 1 : 0);
  if (c->p.q == 19)
    hipLaunchKernelGGL(k_bub_union<19>, grid, block, 0, s, c->d, force ? 1 : 0);
  else
    hipLaunchKernelGGL(k_bub_union<27>, grid, block, 0, s, c->d, force ? 1 : 0);
  const dim3 walk((unsigned)bub_walk_blocks(c->L.N));
  hipLaunchKernelGGL(k_bub_volume, walk, block, 0, s, c->d);
  hipLaunchKernelGGL(k_bub_amount, walk, block, 0, s, c->d);
  hipLaunchKernelGGL(k_bub_target, grid, block, 0, s, c->d);
  hipLaunchKernelGGL(k_bub_pressure, grid, block, 0, s, c->d);
  hipLaunchKernelGGL(k_bub_cells, grid, block, 0, s, c->d);
}

void enqueue_plain(fslbm_ctx* c, int64_t n) {
  const Ops ops = pick(c->p);
  hipStream_t s = c->stream;
  const bool st = c->p.sigma != 0.0;
  for (int64_t i = 0; i < n; ++i) {
    c->d.step = c->step;
    if (st) {
      hipLaunchKernelGGL(k_smooth_mark, dim3(list_blocks(c)), dim3(kBlock), 0, s, c->d);
      hipLaunchKernelGGL(k_smooth, dim3((unsigned)(((c->p.nx + 63) / 64) * ((c->p.ny + 3) / 4) *
                                                   c->p.nz)),
                         dim3(kBlock), 0, s, c->d);
      hipLaunchKernelGGL(k_curvature, dim3(curv_blocks(c)), dim3(kBlock), 0, s, c->d);
    }
    ops.step(c, s);
    ops.convert(c, s, 0);
    if (c->p.bubble_model == 1) launch_volume(c, s, false);
    if (c->p.bubble_model == 2) launch_bubbles(c, s, false);
    std::swap(c->d.fA, c->d.fB);
    std::swap(c->d.phiA, c->d.phiB);
    c->step += 1;
  }
}

void drop_graph(fslbm_ctx* c) {
  for (int li = 0; li < 2; ++li)
    for (int par = 0; par < 2; ++par) {
      if (c->graph_exec[li][par]) (void)hipGraphExecDestroy(c->graph_exec[li][par]);
      if (c->graph[li][par]) (void)hipGraphDestroy(c->graph[li][par]);
      c->graph_exec[li][par] = nullptr;
      c->graph[li][par] = nullptr;
    }
}

constexpr int64_t kGraphLen[2] = {kGraphSteps, 2};

// Captures (without running) the launches of kGraphLen[li] steps starting at
// step parity `par` as a graph and instantiates it. Recording the steps
// advances the host-side step counter and swaps the buffer pointers an even
// number of times, so both end where they started; for the other parity the
// host view is first moved one step on (counter and pointers, nothing runs)
// and moved back afterwards.
int capture_graph(fslbm_ctx* c, int li, int par) {
  hipStream_t s = c->stream;
  const bool flip = (int)(c->step & 1) != par;
  auto turn = [&](int64_t d) {
    c->step += d;
    std::swap(c->d.fA, c->d.fB);
    std::swap(c->d.phiA, c->d.phiB);
  };
  if (flip) turn(1);
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed);
  if (e == hipSuccess) {
    enqueue_plain(c, kGraphLen[li]);
    c->step -= kGraphLen[li];
    e = hipStreamEndCapture(s, &c->graph[li][par]);
    if (e == hipSuccess) e = hipGraphInstantiate(&c->graph_exec[li][par], c->graph[li][par], nullptr, nullptr, 0);
  }
  if (flip) turn(-1);
  if (e != hipSuccess) return hip_fail(c, e, "step graph capture");
  return FSLBM_OK;
}

bool graphs_usable(const fslbm_ctx* c) { return c->graphs && c->ev.empty() && c->stream != nullptr; }

// Every graph a run can replay, captured now (so that no later step of a
// timed region pays for a capture).
int capture_all(fslbm_ctx* c) {
  for (int li = 0; li < 2; ++li)
    for (int par = 0; par < 2; ++par)
      if (!c->graph_exec[li][par]) {
        const int st = capture_graph(c, li, par);
        if (st != FSLBM_OK) return st;
      }
  return FSLBM_OK;
}

// Steps go to the stream as replayed graphs of kGraphSteps steps, then of 2
// steps, where possible (one launch instead of ~5 per step); an odd last step
// as plain launches. Timing runs (events per streaming launch) always use
// plain launches.
int enqueue_steps(fslbm_ctx* c, int64_t n) {
  hipStream_t s = c->stream;
  const bool use_graph = graphs_usable(c);
  while (use_graph && n >= 2) {
    const int li = n >= kGraphSteps ? 0 : 1;
    const int par = (int)(c->step & 1);
    if (!c->graph_exec[li][par]) {
      const int st = capture_graph(c, li, par);
      if (st != FSLBM_OK) return st;
    }
    c->step += kGraphLen[li];  // pointers are back where they were captured
    hipError_t e = hipGraphLaunch(c->graph_exec[li][par], s);
    if (e != hipSuccess) return hip_fail(c, e, "hipGraphLaunch");
    n -= kGraphLen[li];
  }
  enqueue_plain(c, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(c, e, "kernel launch");
  return FSLBM_OK;
}

int read_status(fslbm_ctx* c) {
  int32_t cnt[CNT_N];
  HIPCHK(c, hipMemcpyAsync(cnt, c->d.cnt, sizeof cnt, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const int err = cnt[CNT_ERR];
  if (err & ERR_SCAN) {
    c->status = FSLBM_EDEVICE;
    return set_err(c, FSLBM_EDEVICE, "interface-list scan did not complete");
  }
  if (err & ERR_BUBBLE) {
    c->status = FSLBM_EDEVICE;
    return set_err(c, FSLBM_EDEVICE, "bubble labelling did not complete");
  }
  if (err & ERR_STASH) {
    char buf[200];
    snprintf(buf, sizeof buf,
             "in-place layout: more interface cells than a stash buffer holds (%lld) by step %lld; the "
             "run stopped",
             (long long)c->L.stash_cap, (long long)c->step);
    return set_err(c, FSLBM_ENOMEM, buf);
  }
  if (err & (ERR_UNSTABLE | ERR_LAYER)) {
    char buf[160];
    snprintf(buf, sizeof buf, "instability detected by step %lld (%s)", (long long)c->step,
             (err & ERR_LAYER) ? "liquid cell next to gas" : "NaN, rho <= 0 or |u| >= c_s");
    return set_err(c, FSLBM_EUNSTABLE, buf);
  }
  return FSLBM_OK;
}

}  // namespace

extern "C" {

int fslbm_workspace_bytes(const fslbm_params* p, size_t* bytes) {
  if (!bytes) return FSLBM_EINVAL;
  const char* why = validate(p);
  if (why) {
    snprintf(g_create_error, sizeof g_create_error, "%s", why);
    return FSLBM_EINVAL;
  }
  *bytes = make_layout(*p).total;
  return FSLBM_OK;
}

int fslbm_create(const fslbm_params* p, const uint8_t* type, const double* phi, const double* rho,
                 const double* ux, const double* uy, const double* uz, const double* pdf_or_null,
                 const double* mass_or_null, void* device_arena_or_null, size_t arena_bytes,
                 void* hip_stream, fslbm_ctx** out) {
  if (!out) return FSLBM_EINVAL;
  *out = nullptr;
  const char* why = validate(p);
  if (!why && (!type || !phi || !rho || !ux || !uy || !uz)) why = "field pointer is NULL";
  if (why) {
    snprintf(g_create_error, sizeof g_create_error, "%s", why);
    return FSLBM_EINVAL;
  }
  fslbm_ctx* c = new (std::nothrow) fslbm_ctx();
  if (!c) return FSLBM_ENOMEM;
  c->p = *p;
  c->L = make_layout(*p);
  c->stream = static_cast<hipStream_t>(hip_stream);
  if (device_arena_or_null) {
    if (arena_bytes < c->L.total) {
      snprintf(g_create_error, sizeof g_create_error, "arena of %zu bytes, %zu needed", arena_bytes,
               c->L.total);
      delete c;
      return FSLBM_ENOMEM;
    }
    c->arena = static_cast<char*>(device_arena_or_null);
  } else {
    void* a = nullptr;
    if (hipMalloc(&a, c->L.total) != hipSuccess) {
      (void)hipGetLastError();
      snprintf(g_create_error, sizeof g_create_error, "hipMalloc of %zu bytes failed", c->L.total);
      delete c;
      return FSLBM_ENOMEM;
    }
    c->arena = static_cast<char*>(a);
    c->own_arena = true;
  }
  bind(c);
  {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
      c->device = dev;
      if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
        c->cus = cus;
      // set-up of fslbm_mass_noalloc on this device (its scratch address)
      (void)scratch_for_current_device(dev);
    }
    (void)hipGetLastError();
  }
  const Ops ops = pick(c->p);
  hipStream_t s = c->stream;
  const int64_t N = c->L.N;
  auto fail = [&](int st) {
    snprintf(g_create_error, sizeof g_create_error, "%s", c->last_error.c_str());
    fslbm_destroy(c);
    return st;
  };
#define INITCHK(expr)                                      \
  do {                                                     \
    hipError_t e_ = (expr);                                \
    if (e_ != hipSuccess) return fail(hip_fail(c, e_, #expr)); \
  } while (0)
  {
    int32_t cnt0[CNT_N] = {0};
    cnt0[CNT_EPOCH] = 1;  // status arrays start at epoch 0
    INITCHK(hipMemcpyAsync(c->d.cnt, cnt0, sizeof cnt0, hipMemcpyHostToDevice, s));
    INITCHK(hipStreamSynchronize(s));
  }
  INITCHK(hipMemsetAsync(c->d.scan_status, 0, 16 * c->L.tiles, s));
  if (c->d.smap)  // no smoothing tile is tagged (tags start at 1)
    INITCHK(hipMemsetAsync(c->d.smap, 0, 4 * (size_t)smooth_tiles(c->p.nx, c->p.ny, c->p.nz), s));
  INITCHK(hipMemsetAsync(c->d.fB, 0, (size_t)c->p.q * c->L.stride * storage_bytes(c->p.storage), s));
  // types go straight into the flag array, fields into buffers used as staging
  INITCHK(hipMemcpyAsync(c->d.flags, type, N, hipMemcpyHostToDevice, s));
  INITCHK(hipMemcpyAsync(c->d.phiA, phi, 8 * N, hipMemcpyHostToDevice, s));
  INITCHK(hipMemcpyAsync(c->d.rho_if, rho, 8 * N, hipMemcpyHostToDevice, s));
  INITCHK(hipMemcpyAsync(c->d.m, ux, 8 * N, hipMemcpyHostToDevice, s));
  INITCHK(hipMemcpyAsync(c->d.lost, uy, 8 * N, hipMemcpyHostToDevice, s));
  INITCHK(hipMemcpyAsync(c->d.phiB, uz, 8 * N, hipMemcpyHostToDevice, s));
  ops.init_flags(c, s);
  hipLaunchKernelGGL(k_apply_border, dim3(grid_for(N)), dim3(kBlock), 0, s, c->d);
  if (c->d.aa) {
    // every slot of the in-place layout has one (cell, direction) pair
    const size_t words = ((size_t)c->p.q * c->L.stride + 31) / 32;
    INITCHK(hipMemsetAsync(stage(c), 0, 4 * words, s));
    ops.aa_check(c, s, reinterpret_cast<uint32_t*>(stage(c)));
  }
  int32_t cnt[CNT_N];
  INITCHK(hipMemcpyAsync(cnt, c->d.cnt, sizeof cnt, hipMemcpyDeviceToHost, s));
  INITCHK(hipStreamSynchronize(s));
  if (cnt[CNT_ERR] & ERR_TYPE) {
    c->last_error = "unknown cell type in the initial types";
    return fail(FSLBM_EINVAL);
  }
  if (cnt[CNT_ERR] & ERR_LAYER) {
    c->last_error = "a liquid cell touches a gas cell: the interface layer is not closed";
    return fail(FSLBM_EINVAL);
  }
  if (cnt[CNT_ERR] & ERR_SLOTS) {
    c->last_error =
        "in-place layout: with these walls and obstacles pull streaming takes some population twice "
        "(free-slip faces or obstacles meeting other obstacles); use FSLBM_TWO_GRID";
    return fail(FSLBM_EINVAL);
  }
  const bool resume = pdf_or_null != nullptr;
  if (resume) {
    for (int k = 0; k < c->p.q; ++k) {
      INITCHK(hipMemcpyAsync(stage(c), pdf_or_null + (size_t)k * N, 8 * N, hipMemcpyHostToDevice, s));
      ops.import_plane(c, s, stage(c), k);
    }
  }
  ops.init_state(c, s, resume ? 1 : 0);
  if (resume && mass_or_null) {
    // interface mass verbatim; liquid/gas entries are ignored by the step
    INITCHK(hipMemcpyAsync(c->d.m, mass_or_null, 8 * N, hipMemcpyHostToDevice, s));
  }
  // interface list, flux classes, volume pressure
  c->d.step = 0;
  ops.convert(c, s, 1);
  ops.classes(c, s);
  if (c->d.aa) ops.stash_init(c, s);  // the interface cells' own populations
  const double pv0[3] = {c->p.rho_gas / 3.0, c->p.rho_gas / 3.0, 0.0};
  INITCHK(hipMemcpyAsync(c->d.pV, pv0, sizeof pv0, hipMemcpyHostToDevice, s));
  // V(0) from phiB == phiA at this point
  launch_volume(c, s, true);
  if (c->p.bubble_model == 2) {
    // no old bubbles: every bubble starts at p^V(0)
    INITCHK(hipMemsetAsync(c->d.blab, 0xff, 4 * N, s));
    launch_bubbles(c, s, true);
  }
  INITCHK(hipGetLastError());
  INITCHK(hipStreamSynchronize(s));
  if (c->d.aa) {
    INITCHK(hipMemcpyAsync(cnt, c->d.cnt, sizeof cnt, hipMemcpyDeviceToHost, s));
    INITCHK(hipStreamSynchronize(s));
    if (cnt[CNT_ERR] & ERR_STASH) {
      char buf[160];
      snprintf(buf, sizeof buf, "in-place layout: more interface cells than a stash buffer holds (%lld)",
               (long long)c->L.stash_cap);
      c->last_error = buf;
      return fail(FSLBM_ENOMEM);
    }
  }
#undef INITCHK
  *out = c;
  return FSLBM_OK;
}

int fslbm_set_variant(fslbm_ctx* c, int variant) {
  if (!c) return FSLBM_EINVAL;
  if (variant < FSLBM_NBRC || variant > FSLBM_OM3) return set_err(c, FSLBM_EINVAL, "unknown variant");
  c->p.variant = variant;
  c->d.variant = variant;
  drop_graph(c);  // the variant is a kernel argument of the captured launches
  return FSLBM_OK;
}

int fslbm_step(fslbm_ctx* c, int64_t nsteps) {
  if (!c) return FSLBM_EINVAL;
  if (nsteps < 0) return set_err(c, FSLBM_EINVAL, "nsteps < 0");
  if (c->status != FSLBM_OK) return set_err(c, FSLBM_ESTATE, "context failed earlier: " + c->last_error);
  return enqueue_steps(c, nsteps);
}

int fslbm_mass(fslbm_ctx* c, fslbm_mass_report* r) {
  if (!c || !r) return FSLBM_EINVAL;
  if (c->status != FSLBM_OK) return set_err(c, FSLBM_ESTATE, "context failed earlier: " + c->last_error);
  c->d.step = c->step;  // kernels below read the state before step c->step
  const Ops ops = pick(c->p);
  hipStream_t s = c->stream;
  ops.reduce_mass(c->d, c->L.red_blocks, s);
  double* out = c->d.partial + kRedN * c->L.red_blocks;
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, s, c->d.partial, (int)c->L.red_blocks,
                     kRedN, out);
  double v[kRedN], pv[3];
  HIPCHK(c, hipMemcpyAsync(v, out, sizeof v, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipMemcpyAsync(pv, c->d.pV, sizeof pv, hipMemcpyDeviceToHost, s));
  const int st = read_status(c);
  if (st == FSLBM_EDEVICE) return st;
  r->liquid_mass = v[0];
  r->interface_mass = v[1];
  r->lost_mass = v[2];
  r->total_mass = v[0] + v[1] + v[2];
  r->bubble_volume = v[3];
  r->p_volume = pv[0];
  r->n_liquid = (int64_t)v[4];
  r->n_interface = (int64_t)v[5];
  r->n_gas = (int64_t)v[6];
  r->step = c->step;
  return st;
}

int fslbm_mass_noalloc(fslbm_ctx* c, double* out_device) {
  if (!c || !out_device) return FSLBM_EINVAL;
  if (c->status != FSLBM_OK) return set_err(c, FSLBM_ESTATE, "context failed earlier: " + c->last_error);
  if (c->L.red_blocks > kNoAllocBlocks) {
    char buf[200];
    snprintf(buf, sizeof buf,
             "fslbm_mass_noalloc: %lld cells exceed its scratch (at most %lld cells); use fslbm_mass",
             (long long)c->L.N, (long long)(kNoAllocBlocks * kRedCells));
    return set_err(c, FSLBM_EINVAL, buf);
  }
  double* scr = (c->device >= 0 && c->device < kMaxDevices) ? g_scratch[c->device] : nullptr;
  if (!scr) return set_err(c, FSLBM_EDEVICE, "fslbm_mass_noalloc: scratch address not resolved");
  const Ops ops = pick(c->p);
  hipStream_t s = c->stream;
  // the reduction of fslbm_mass (same blocks, same order), partials in the scratch
  Dev d = c->d;  // (a plain struct of pointers and numbers: no allocation)
  d.step = c->step;  // the state before step c->step
  d.partial = scr;
  ops.reduce_mass(d, c->L.red_blocks, s);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, s, scr, (int)c->L.red_blocks, kRedN,
                     out_device + 1);
  hipLaunchKernelGGL(k_total_of_report, dim3(1), dim3(64), 0, s, out_device);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(c, e, "fslbm_mass_noalloc launch");
  return FSLBM_OK;
}

int fslbm_fields(fslbm_ctx* c, uint8_t* type, double* phi, double* rho, double* ux, double* uy,
                 double* uz, double* mass, double* pdf) {
  if (!c) return FSLBM_EINVAL;
  if (c->status != FSLBM_OK) return set_err(c, FSLBM_ESTATE, "context failed earlier: " + c->last_error);
  c->d.step = c->step;  // kernels below read the state before step c->step
  const Ops ops = pick(c->p);
  hipStream_t s = c->stream;
  const int64_t N = c->L.N;
  double* st = stage(c);
  if (type) {
    std::vector<uint8_t> fl(N);
    HIPCHK(c, hipMemcpyAsync(fl.data(), c->d.flags, N, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    for (int64_t i = 0; i < N; ++i) type[i] = fl[i] & T_MASK;
  }
  double* outs[6] = {rho, ux, uy, uz, mass, phi};
  for (int w = 0; w < 6; ++w) {
    if (!outs[w]) continue;
    ops.export_field(c, s, st, w);
    HIPCHK(c, hipMemcpyAsync(outs[w], st, 8 * N, hipMemcpyDeviceToHost, s));
  }
  if (pdf) {
    for (int k = 0; k < c->p.q; ++k) {
      ops.export_field(c, s, st, 10 + k);
      HIPCHK(c, hipMemcpyAsync(pdf + (size_t)k * N, st, 8 * N, hipMemcpyDeviceToHost, s));
    }
  }
  HIPCHK(c, hipGetLastError());
  return read_status(c);
}

int fslbm_interface_list(fslbm_ctx* c, int32_t* list, int64_t max, int64_t* count) {
  if (!c || !count) return FSLBM_EINVAL;
  int32_t cnt[CNT_N];
  HIPCHK(c, hipMemcpyAsync(cnt, c->d.cnt, sizeof cnt, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  *count = cnt[CNT_IF];
  if (list && max > 0) {
    const int64_t n = std::min<int64_t>(max, cnt[CNT_IF]);
    HIPCHK(c, hipMemcpyAsync(list, c->d.if_list, 4 * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int64_t i = 0; i < n; ++i) list[i] &= 0x7fffffff;  // drop the BORDER bit
  }
  return FSLBM_OK;
}

int fslbm_bubbles(fslbm_ctx* c, int64_t* label, double* volume, double* pressure, int64_t max,
                  int64_t* count) {
  if (!c || !count) return FSLBM_EINVAL;
  *count = 0;
  if (max > 0 && (!label || !volume || !pressure)) return set_err(c, FSLBM_EINVAL, "NULL output array");
  if (c->p.bubble_model != 2) return FSLBM_OK;
  const int64_t N = c->L.N;
  std::vector<int32_t> lab(N);
  std::vector<double> P(N);
  std::vector<int64_t> Vh(N);
  std::vector<uint64_t> Vl(N);
  HIPCHK(c, hipMemcpyAsync(lab.data(), c->d.blab, 4 * N, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(Vh.data(), c->d.bV, 8 * N, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(Vl.data(), c->d.bVl, 8 * N, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(P.data(), c->d.bpr, 8 * N, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  int64_t n = 0;
  for (int64_t i = 0; i < N; ++i) {
    if (lab[i] != (int32_t)i) continue;
    if (n < max) {
      label[n] = i;
      volume[n] = fix_value(Vh[i], Vl[i]);
      pressure[n] = P[i];
    }
    ++n;
  }
  *count = n;
  return read_status(c);
}

static void release_events(fslbm_ctx* c) {
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  c->ev.clear();
  c->ev_used = 0;
}

int fslbm_set_graphs(fslbm_ctx* c, int enable) {
  if (!c) return FSLBM_EINVAL;
  c->graphs = enable != 0;
  if (!c->graphs) {
    drop_graph(c);
    return FSLBM_OK;
  }
  if (c->status != FSLBM_OK) return set_err(c, FSLBM_ESTATE, "context failed earlier: " + c->last_error);
  // capture now, so that the first steps replay instead of capturing
  if (graphs_usable(c)) return capture_all(c);
  return FSLBM_OK;
}

int fslbm_set_compaction_tile(fslbm_ctx* c, int cells_per_thread) {
  if (!c) return FSLBM_EINVAL;
  const int64_t per = cells_per_thread;
  const bool pow2 = per >= 16 && per % 16 == 0 && ((per / 16) & (per / 16 - 1)) == 0;
  if (!pow2 || per < c->L.conv_per || per > 4096) return FSLBM_EINVAL;
  // fewer tiles than the status array was sized for
  c->L.conv_per = per;
  c->L.tiles = (c->L.N + (int64_t)kCompBlock * per - 1) / ((int64_t)kCompBlock * per);
  drop_graph(c);  // the tile count and size are launch arguments of the captured steps
  return FSLBM_OK;
}

int fslbm_set_timing(fslbm_ctx* c, int64_t capacity) {
  if (!c || capacity < 0) return FSLBM_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  release_events(c);
  c->ev.reserve((size_t)(2 * capacity));
  // timing only: no system-scope fence when an event completes (its cache
  // write-back and invalidation would slow the launches being timed; the
  // stream synchronisation before the times are read orders them)
  for (int64_t i = 0; i < 2 * capacity; ++i) {
    hipEvent_t e;
    HIPCHK(c, hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    c->ev.push_back(e);
  }
  return FSLBM_OK;
}

int fslbm_kernel_time(fslbm_ctx* c, int64_t* launches, double* total_ms) {
  if (!c || !launches || !total_ms) return FSLBM_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double t = 0.0;
  for (int64_t i = 0; i < c->ev_used; ++i) {
    float ms = 0.0f;
    HIPCHK(c, hipEventElapsedTime(&ms, c->ev[2 * i], c->ev[2 * i + 1]));
    t += ms;
  }
  *launches = c->ev_used;
  *total_ms = t;
  return FSLBM_OK;
}

int fslbm_get_scalars(fslbm_ctx* c, double out[4]) {
  if (!c || !out) return FSLBM_EINVAL;
  if (c->status != FSLBM_OK) return set_err(c, FSLBM_ESTATE, "context failed earlier: " + c->last_error);
  c->d.step = c->step;  // kernels below read the state before step c->step
  const Ops ops = pick(c->p);
  hipStream_t s = c->stream;
  ops.reduce_mass(c->d, c->L.red_blocks, s);
  double* red = c->d.partial + kRedN * c->L.red_blocks;
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, s, c->d.partial, (int)c->L.red_blocks,
                     kRedN, red);
  double v[kRedN], pv[3];
  HIPCHK(c, hipMemcpyAsync(v, red, sizeof v, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipMemcpyAsync(pv, c->d.pV, sizeof pv, hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  out[0] = v[2];
  out[1] = pv[0];
  out[2] = pv[1];
  out[3] = pv[2];
  return FSLBM_OK;
}

int fslbm_set_scalars(fslbm_ctx* c, const double in[4]) {
  if (!c || !in) return FSLBM_EINVAL;
  if (c->status != FSLBM_OK) return set_err(c, FSLBM_ESTATE, "context failed earlier: " + c->last_error);
  for (int i = 0; i < 4; ++i)
    if (!std::isfinite(in[i])) return set_err(c, FSLBM_EINVAL, "non-finite scalar");
  if (!(in[3] > 0.0) && c->p.bubble_model == 1) return set_err(c, FSLBM_EINVAL, "V(0) must be > 0");
  hipStream_t s = c->stream;
  // the lost mass is kept per cell and summed when reported: the whole
  // restored amount goes to the first cell's entry
  HIPCHK(c, hipMemsetAsync(c->d.lost, 0, 8 * c->L.N, s));
  HIPCHK(c, hipMemcpyAsync(c->d.lost, &in[0], sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(c->d.pV, &in[1], 3 * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(c, hipStreamSynchronize(s));
  return FSLBM_OK;
}

void fslbm_destroy(fslbm_ctx* c) {
  if (!c) return;
  if (c->arena) {
    (void)hipStreamSynchronize(c->stream);
    if (c->own_arena) (void)hipFree(c->arena);
  }
  release_events(c);
  drop_graph(c);
  delete c;
}

const char* fslbm_strerror(int status) {
  switch (status) {
    case FSLBM_OK: return "ok";
    case FSLBM_EINVAL: return "invalid argument";
    case FSLBM_ENOMEM: return "out of device memory";
    case FSLBM_EDEVICE: return "device error";
    case FSLBM_EUNSTABLE: return "simulation unstable";
    case FSLBM_ESTATE: return "invalid state";
    case FSLBM_EBUDGET: return "request exceeds the memory budget";
    default: return "unknown status";
  }
}

const char* fslbm_last_error(const fslbm_ctx* c) {
  if (!c) return g_create_error;
  return c->last_error.c_str();
}

}  // extern "C"

// ===========================================================================
// Serving: runs of a batch share each step launch (see include/fslbm.h).
// ===========================================================================
namespace {

// First-fit allocator over the server's device pool, 256-byte granules.
class Pool {
 public:
  explicit Pool(size_t size) : size_(size) { free_.push_back({0, size}); }
  bool alloc(size_t bytes, size_t* off) {
    bytes = (size_t)round_up((int64_t)bytes, 256);
    for (size_t i = 0; i < free_.size(); ++i) {
      if (free_[i].size < bytes) continue;
      *off = free_[i].off;
      free_[i].off += bytes;
      free_[i].size -= bytes;
      if (free_[i].size == 0) free_.erase(free_.begin() + (long)i);
      used_ += bytes;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (size_t)round_up((int64_t)bytes, 256);
    used_ -= bytes;
    auto it = std::lower_bound(free_.begin(), free_.end(), off,
                               [](const Span& a, size_t o) { return a.off < o; });
    it = free_.insert(it, {off, bytes});
    // coalesce with the neighbours
    const size_t i = (size_t)(it - free_.begin());
    if (i + 1 < free_.size() && free_[i].off + free_[i].size == free_[i + 1].off) {
      free_[i].size += free_[i + 1].size;
      free_.erase(free_.begin() + (long)i + 1);
    }
    if (i > 0 && free_[i - 1].off + free_[i - 1].size == free_[i].off) {
      free_[i - 1].size += free_[i].size;
      free_.erase(free_.begin() + (long)i);
    }
  }
  size_t used() const { return used_; }
  size_t size() const { return size_; }

 private:
  struct Span {
    size_t off, size;
  };
  size_t size_, used_ = 0;
  std::vector<Span> free_;
};

struct PendingRun {
  uint64_t id;
  fslbm_params p;
  std::vector<uint8_t> type;
  std::vector<double> phi, rho, ux, uy, uz;
  int64_t nsteps;
  size_t bytes;
};

struct ResidentRun {
  uint64_t id;
  fslbm_ctx* ctx;
  size_t off, bytes;
  int64_t tick0, nsteps;
  int slot, group;
};

struct DoneRun {
  int status;
  fslbm_mass_report rep;
  std::vector<double> phi;
};

// launch groups: storage (3) x lattice (2) x collision (2) x layout (2) x addressing (2)
constexpr int kGroups = 48;

int group_of(const fslbm_params& p, bool buf) {
  return (((p.storage * 2 + (p.q == 27 ? 1 : 0)) * 2 + (p.collision == FSLBM_TRT ? 1 : 0)) * 2 +
          (p.layout == FSLBM_AA ? 1 : 0)) * 2 + (buf ? 1 : 0);
}

bool grid_fits_buffer(const fslbm_ctx* c) {
  return (double)c->p.q * (double)c->L.stride * storage_bytes(c->p.storage) < 2147483648.0;
}

int round8(int64_t b) { return (int)std::max<int64_t>(kXcds, (b + kXcds - 1) / kXcds * kXcds); }

}  // namespace

struct fslbm_server {
  size_t budget = 0;
  int max_slots = 0;
  hipStream_t stream = nullptr;
  char* pool_mem = nullptr;
  Pool* pool = nullptr;
  Dev* d_devs = nullptr;          // max_slots Dev records
  BatchEntry* d_tab = nullptr;    // kGroups x kLaunches x max_slots entries
  BatchEntry* h_tab = nullptr;    // pinned staging of the same
  std::vector<int> free_slots;
  std::deque<PendingRun> queue;
  std::vector<ResidentRun> resident;
  std::map<uint64_t, DoneRun> done;
  std::vector<std::pair<uint64_t, int>> unpolled;
  BatchLaunch launch[kGroups];
  // groups touch disjoint runs: each runs its ticks on a stream of its own
  // (default priority), forked from and joined back to `stream` per chunk
  static constexpr int kGroupStreams = 4;
  hipStream_t gstream[kGroupStreams] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[kGroupStreams] = {nullptr, nullptr, nullptr, nullptr};
  bool dirty = true;
  uint64_t next_id = 1;
  int64_t tick = 0, completed = 0;
  size_t peak = 0;
  int status = FSLBM_OK;
};

namespace {

int srv_fail(fslbm_server* s, hipError_t e) {
  (void)e;
  s->status = FSLBM_EDEVICE;
  return FSLBM_EDEVICE;
}

// Block ranges of one run in the launches of a batched step.
void run_blocks(const fslbm_ctx* c, int nb[kLaunches], int stream_split[2], int compact_args[2]) {
  const int gen = round8(std::min<int64_t>(if_blocks(c), 192));
  const int bord = round8(std::min<int64_t>(border_blocks(c), 64));
  const int liq = round8(std::min<int64_t>(liquid_blocks(c), 256));
  stream_split[0] = gen;
  stream_split[1] = bord;
  nb[0] = gen + bord + liq;
  // (only the streaming launch needs XCD-aligned ranges; the compaction needs
  // exactly one block per tile beside its workers)
  nb[1] = (int)std::min<int64_t>(retype_blocks(c), 64);
  const int workers = compact_workers(c);
  compact_args[0] = (int)c->L.conv_per;
  compact_args[1] = workers;
  nb[2] = (int)c->L.tiles + workers;
}

// Tables of every group from the resident runs.
int rebuild_plan(fslbm_server* s) {
  if (hipStreamSynchronize(s->stream) != hipSuccess) return srv_fail(s, hipErrorUnknown);
  for (int g = 0; g < kGroups; ++g) {
    BatchLaunch& bl = s->launch[g];
    bl = BatchLaunch{};
    bl.devs = s->d_devs;
    bl.buf = (g & 1) != 0;
    bl.aa = (g & 2) != 0;
    bl.q = ((g >> 3) & 1) != 0 ? 27 : 19;
    int cursor[kLaunches] = {0, 0, 0};
    int xcursor[kAux] = {};
    for (const ResidentRun& r : s->resident) {
      if (r.group != g) continue;
      // the launches beside the step, for the runs that need them
      const fslbm_ctx* c = r.ctx;
      const bool st = c->p.sigma != 0.0, bub = c->p.bubble_model == 1, tracked = c->p.bubble_model == 2;
      const int64_t xnb[kAux] = {smooth_tiles(c->p.nx, c->p.ny, c->p.nz), std::min<int64_t>(curv_blocks(c), 128),
                                 vol_blocks_of(c->L.N), 1, grid_for(c->L.N), bub_walk_blocks(c->L.N)};
      for (int k = 0; k < kAux; ++k) {
        if (!(k < AUX_VOL ? st : (k < AUX_BUB ? bub : tracked))) continue;
        BatchEntry& e = s->h_tab[((size_t)g * kTabs + kLaunches + k) * s->max_slots + bl.aux_n[k]];
        e.slot = r.slot;
        e.blk0 = xcursor[k];
        e.nblk = (int32_t)xnb[k];
        e.a = e.b = e.pad = 0;
        e.tick0 = r.tick0;
        e.nsteps = r.nsteps;
        xcursor[k] += (int)xnb[k];
        ++bl.aux_n[k];
      }
      int nb[kLaunches], split[2], cargs[2];
      run_blocks(r.ctx, nb, split, cargs);
      for (int k = 0; k < kLaunches; ++k) {
        BatchEntry& e = s->h_tab[((size_t)g * kTabs + k) * s->max_slots + bl.n];
        e.slot = r.slot;
        e.blk0 = cursor[k];
        e.nblk = nb[k];
        e.a = k == 0 ? split[0] : (k == 2 ? cargs[0] : 0);
        e.b = k == 0 ? split[1] : (k == 2 ? cargs[1] : 0);
        e.pad = 0;
        e.tick0 = r.tick0;
        e.nsteps = r.nsteps;
        cursor[k] += nb[k];
      }
      ++bl.n;
    }
    for (int k = 0; k < kLaunches; ++k) {
      const size_t at = ((size_t)g * kTabs + k) * s->max_slots;
      bl.blocks[k] = cursor[k];
      bl.tab[k] = s->d_tab + at;
      if (bl.n > 0 && hipMemcpyAsync(const_cast<BatchEntry*>(bl.tab[k]), s->h_tab + at, sizeof(BatchEntry) * bl.n,
                                     hipMemcpyHostToDevice, s->stream) != hipSuccess)
        return srv_fail(s, hipErrorUnknown);
    }
    for (int k = 0; k < kAux; ++k) {
      const size_t at = ((size_t)g * kTabs + kLaunches + k) * s->max_slots;
      bl.aux_blocks[k] = xcursor[k];
      bl.aux[k] = s->d_tab + at;
      if (bl.aux_n[k] > 0 &&
          hipMemcpyAsync(const_cast<BatchEntry*>(bl.aux[k]), s->h_tab + at, sizeof(BatchEntry) * bl.aux_n[k],
                         hipMemcpyHostToDevice, s->stream) != hipSuccess)
        return srv_fail(s, hipErrorUnknown);
    }
  }
  s->dirty = false;
  return FSLBM_OK;
}

// Runs that have taken all their steps: results out, memory and slot back.
int retire_finished(fslbm_server* s) {
  bool any = false;
  for (const ResidentRun& r : s->resident) any |= s->tick >= r.tick0 + r.nsteps;
  if (!any) return FSLBM_OK;
  if (hipStreamSynchronize(s->stream) != hipSuccess) return srv_fail(s, hipErrorUnknown);
  std::vector<ResidentRun> keep;
  for (ResidentRun& r : s->resident) {
    if (s->tick < r.tick0 + r.nsteps) {
      keep.push_back(r);
      continue;
    }
    fslbm_ctx* c = r.ctx;
    // the host view of a single run after nsteps steps
    c->step = r.nsteps;
    if (r.nsteps & 1) {
      std::swap(c->d.fA, c->d.fB);
      std::swap(c->d.phiA, c->d.phiB);
    }
    DoneRun dr;
    dr.status = fslbm_mass(c, &dr.rep);
    if (dr.status == FSLBM_EDEVICE) return srv_fail(s, hipErrorUnknown);
    dr.phi.resize((size_t)c->L.N);
    const int fs = fslbm_fields(c, nullptr, dr.phi.data(), nullptr, nullptr, nullptr, nullptr, nullptr,
                                nullptr);
    if (fs == FSLBM_EDEVICE) return srv_fail(s, hipErrorUnknown);
    if (dr.status == FSLBM_OK) dr.status = fs;
    fslbm_destroy(c);
    s->pool->release(r.off, r.bytes);
    s->free_slots.push_back(r.slot);
    s->unpolled.push_back({r.id, dr.status});
    s->done[r.id] = std::move(dr);
    ++s->completed;
  }
  s->resident.swap(keep);
  s->dirty = true;
  return FSLBM_OK;
}

// Queued runs, in order, while a slot and pool memory are free.
int admit_queued(fslbm_server* s) {
  while (!s->queue.empty() && !s->free_slots.empty()) {
    PendingRun& q = s->queue.front();
    size_t off;
    if (!s->pool->alloc(q.bytes, &off)) break;
    fslbm_ctx* c = nullptr;
    const int st = fslbm_create(&q.p, q.type.data(), q.phi.data(), q.rho.data(), q.ux.data(), q.uy.data(),
                                q.uz.data(), nullptr, nullptr, s->pool_mem + off, q.bytes, s->stream, &c);
    if (st != FSLBM_OK) {
      s->pool->release(off, q.bytes);
      // a run whose initial state is rejected finishes at once with the error
      DoneRun dr;
      dr.status = st;
      std::memset(&dr.rep, 0, sizeof dr.rep);
      s->unpolled.push_back({q.id, st});
      s->done[q.id] = std::move(dr);
      ++s->completed;
      s->queue.pop_front();
      continue;
    }
    ResidentRun r;
    r.id = q.id;
    r.ctx = c;
    r.off = off;
    r.bytes = q.bytes;
    r.tick0 = s->tick;
    r.nsteps = q.nsteps;
    r.slot = s->free_slots.back();
    s->free_slots.pop_back();
    r.group = group_of(c->p, grid_fits_buffer(c));
    if (hipMemcpyAsync(s->d_devs + r.slot, &c->d, sizeof(Dev), hipMemcpyHostToDevice, s->stream) !=
            hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess)
      return srv_fail(s, hipErrorUnknown);
    s->resident.push_back(r);
    s->queue.pop_front();
    s->peak = std::max(s->peak, s->pool->used());
    s->dirty = true;
  }
  return FSLBM_OK;
}

void free_server(fslbm_server* s) {
  for (ResidentRun& r : s->resident) fslbm_destroy(r.ctx);
  for (int k = 0; k < fslbm_server::kGroupStreams; ++k) {
    if (s->gstream[k]) (void)hipStreamSynchronize(s->gstream[k]);
    if (s->gstream[k]) (void)hipStreamDestroy(s->gstream[k]);
    if (s->join_ev[k]) (void)hipEventDestroy(s->join_ev[k]);
  }
  if (s->fork_ev) (void)hipEventDestroy(s->fork_ev);
  if (s->d_devs) (void)hipFree(s->d_devs);
  if (s->d_tab) (void)hipFree(s->d_tab);
  if (s->h_tab) (void)hipHostFree(s->h_tab);
  if (s->pool_mem) (void)hipFree(s->pool_mem);
  delete s->pool;
  delete s;
}

}  // namespace

extern "C" {

int fslbm_server_create(size_t hbm_budget_bytes, int max_slots, void* hip_stream, fslbm_server** out) {
  if (!out) return FSLBM_EINVAL;
  *out = nullptr;
  if (hbm_budget_bytes < 4096 || max_slots < 1 || max_slots > 4096) return FSLBM_EINVAL;
  fslbm_server* s = new (std::nothrow) fslbm_server();
  if (!s) return FSLBM_ENOMEM;
  s->budget = hbm_budget_bytes;
  s->max_slots = max_slots;
  s->stream = static_cast<hipStream_t>(hip_stream);
  const size_t tab = sizeof(BatchEntry) * (size_t)kGroups * kTabs * (size_t)max_slots;
  if (hipMalloc(reinterpret_cast<void**>(&s->pool_mem), hbm_budget_bytes) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&s->d_devs), sizeof(Dev) * (size_t)max_slots) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&s->d_tab), tab) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&s->h_tab), tab, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    free_server(s);
    return FSLBM_ENOMEM;
  }
  s->pool = new (std::nothrow) Pool(hbm_budget_bytes);
  if (!s->pool) {
    free_server(s);
    return FSLBM_ENOMEM;
  }
  bool ok = hipEventCreateWithFlags(&s->fork_ev, hipEventDisableTiming) == hipSuccess;
  for (int k = 0; ok && k < fslbm_server::kGroupStreams; ++k)
    ok = hipStreamCreateWithFlags(&s->gstream[k], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&s->join_ev[k], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    free_server(s);
    return FSLBM_EDEVICE;
  }
  for (int i = max_slots - 1; i >= 0; --i) s->free_slots.push_back(i);
  *out = s;
  return FSLBM_OK;
}

int fslbm_server_submit(fslbm_server* s, const fslbm_params* p, const uint8_t* type, const double* phi,
                        const double* rho, const double* ux, const double* uy, const double* uz,
                        int64_t nsteps, uint64_t* req_id) {
  if (!s || !req_id || !type || !phi || !rho || !ux || !uy || !uz || nsteps <= 0) return FSLBM_EINVAL;
  if (validate(p)) return FSLBM_EINVAL;
  const size_t bytes = make_layout(*p).total;
  if ((size_t)round_up((int64_t)bytes, 256) > s->budget) return FSLBM_EINVAL;
  PendingRun q;
  try {
    const size_t N = (size_t)p->nx * p->ny * p->nz;
    q.type.assign(type, type + N);
    q.phi.assign(phi, phi + N);
    q.rho.assign(rho, rho + N);
    q.ux.assign(ux, ux + N);
    q.uy.assign(uy, uy + N);
    q.uz.assign(uz, uz + N);
  } catch (...) {
    return FSLBM_ENOMEM;
  }
  q.id = s->next_id++;
  q.p = *p;
  q.nsteps = nsteps;
  q.bytes = bytes;
  *req_id = q.id;
  s->queue.push_back(std::move(q));
  return FSLBM_OK;
}

int fslbm_server_advance(fslbm_server* s, int64_t ticks) {
  if (!s || ticks < 0) return FSLBM_EINVAL;
  if (s->status != FSLBM_OK) return s->status;
  int64_t left = ticks;
  for (;;) {
    int st = retire_finished(s);
    if (st != FSLBM_OK) return st;
    st = admit_queued(s);
    if (st != FSLBM_OK) return st;
    if (s->resident.empty() || left <= 0) return FSLBM_OK;
    if (s->dirty && (st = rebuild_plan(s)) != FSLBM_OK) return st;
    // ticks until the next run finishes
    int64_t chunk = left;
    for (const ResidentRun& r : s->resident) chunk = std::min(chunk, r.tick0 + r.nsteps - s->tick);
    // the active groups and their kernel tables
    Ops ops[kGroups];
    int active[kGroups], na = 0;
    for (int g = 0; g < kGroups; ++g) {
      if (s->launch[g].n == 0) continue;
      for (const ResidentRun& r : s->resident)
        if (r.group == g) {
          ops[na] = pick(r.ctx->p);
          break;
        }
      active[na++] = g;
    }
    // one group runs on the server stream; several run side by side on
    // streams of their own (disjoint runs), forked here and joined below
    const bool fork = na > 1;
    int used = 0;
    if (fork) {
      if (hipEventRecord(s->fork_ev, s->stream) != hipSuccess) return srv_fail(s, hipErrorUnknown);
      for (int a = 0; a < na; ++a) used |= 1 << (active[a] % fslbm_server::kGroupStreams);
      for (int k = 0; k < fslbm_server::kGroupStreams; ++k)
        if ((used >> k) & 1)
          if (hipStreamWaitEvent(s->gstream[k], s->fork_ev, 0) != hipSuccess) return srv_fail(s, hipErrorUnknown);
    }
    for (int64_t i = 0; i < chunk; ++i)
      for (int a = 0; a < na; ++a) {
        hipStream_t st = fork ? s->gstream[active[a] % fslbm_server::kGroupStreams] : s->stream;
        const BatchLaunch& bl = s->launch[active[a]];
        const int64_t t = s->tick + i;
        if (bl.aux_n[AUX_SMOOTH] > 0) {
          hipLaunchKernelGGL(kb_smooth, dim3((unsigned)bl.aux_blocks[AUX_SMOOTH]), dim3(kBlock), 0, st, bl.devs,
                             bl.aux[AUX_SMOOTH], bl.aux_n[AUX_SMOOTH], t);
          hipLaunchKernelGGL(kb_curvature, dim3((unsigned)bl.aux_blocks[AUX_CURV]), dim3(kBlock), 0, st, bl.devs,
                             bl.aux[AUX_CURV], bl.aux_n[AUX_CURV], t);
        }
        ops[a].batch_step(bl, st, t);
        if (bl.aux_n[AUX_VOL] > 0) {
          hipLaunchKernelGGL(kb_volume, dim3((unsigned)bl.aux_blocks[AUX_VOL]), dim3(kBlock), 0, st, bl.devs,
                             bl.aux[AUX_VOL], bl.aux_n[AUX_VOL], t);
          hipLaunchKernelGGL(kb_sum_volume, dim3((unsigned)bl.aux_blocks[AUX_SUMVOL]), dim3(kBlock), 0, st,
                             bl.devs, bl.aux[AUX_SUMVOL], bl.aux_n[AUX_SUMVOL], t);
        }
        if (bl.aux_n[AUX_BUB] > 0) {
          const dim3 gc((unsigned)bl.aux_blocks[AUX_BUB]), gw((unsigned)bl.aux_blocks[AUX_BUBW]), b(kBlock);
          const BatchEntry *tc = bl.aux[AUX_BUB], *tw = bl.aux[AUX_BUBW];
          const int nc = bl.aux_n[AUX_BUB], nw = bl.aux_n[AUX_BUBW];
          hipLaunchKernelGGL(kb_bub_init, gc, b, 0, st, bl.devs, tc, nc, t);
          if (bl.q == 19)
            hipLaunchKernelGGL(kb_bub_union<19>, gc, b, 0, st, bl.devs, tc, nc, t);
          else
            hipLaunchKernelGGL(kb_bub_union<27>, gc, b, 0, st, bl.devs, tc, nc, t);
          hipLaunchKernelGGL(kb_bub_volume, gw, b, 0, st, bl.devs, tw, nw, t);
          hipLaunchKernelGGL(kb_bub_amount, gw, b, 0, st, bl.devs, tw, nw, t);
          hipLaunchKernelGGL(kb_bub_target, gc, b, 0, st, bl.devs, tc, nc, t);
          hipLaunchKernelGGL(kb_bub_pressure, gc, b, 0, st, bl.devs, tc, nc, t);
          hipLaunchKernelGGL(kb_bub_cells, gc, b, 0, st, bl.devs, tc, nc, t);
        }
      }
    if (fork) {
      for (int k = 0; k < fslbm_server::kGroupStreams; ++k)
        if ((used >> k) & 1)
          if (hipEventRecord(s->join_ev[k], s->gstream[k]) != hipSuccess ||
              hipStreamWaitEvent(s->stream, s->join_ev[k], 0) != hipSuccess)
            return srv_fail(s, hipErrorUnknown);
    }
    s->tick += chunk;
    if (hipGetLastError() != hipSuccess) return srv_fail(s, hipErrorUnknown);
    left -= chunk;
  }
}

int fslbm_server_poll(fslbm_server* s, uint64_t* done_ids, int* statuses, int max, int* n_done) {
  if (!s || !n_done || max < 0 || (max > 0 && (!done_ids || !statuses))) return FSLBM_EINVAL;
  const int n = (int)std::min<size_t>((size_t)max, s->unpolled.size());
  for (int i = 0; i < n; ++i) {
    done_ids[i] = s->unpolled[(size_t)i].first;
    statuses[i] = s->unpolled[(size_t)i].second;
  }
  s->unpolled.erase(s->unpolled.begin(), s->unpolled.begin() + n);
  *n_done = n;
  return FSLBM_OK;
}

int fslbm_server_result(fslbm_server* s, uint64_t req_id, fslbm_mass_report* report, double* phi_out) {
  if (!s) return FSLBM_EINVAL;
  auto it = s->done.find(req_id);
  if (it == s->done.end()) return FSLBM_EINVAL;
  if (report) *report = it->second.rep;
  if (phi_out && !it->second.phi.empty())
    std::memcpy(phi_out, it->second.phi.data(), sizeof(double) * it->second.phi.size());
  s->done.erase(it);
  return FSLBM_OK;
}

int fslbm_server_stats_get(const fslbm_server* s, fslbm_server_stats* out) {
  if (!s || !out) return FSLBM_EINVAL;
  out->queued = (int64_t)s->queue.size();
  out->resident = (int64_t)s->resident.size();
  out->completed = s->completed;
  out->ticks = s->tick;
  out->bytes_in_use = s->pool->used();
  out->peak_bytes_in_use = s->peak;
  out->budget_bytes = s->budget;
  return FSLBM_OK;
}

void fslbm_server_destroy(fslbm_server* s) {
  if (!s) return;
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  else (void)hipDeviceSynchronize();
  free_server(s);
}

}  // extern "C"
