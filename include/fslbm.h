/*
 * libfslbm - free-surface lattice Boltzmann time step on AMD Instinct MI355X (gfx950).
 *
 * The method is the free-surface lattice Boltzmann method of Schwarzmeier & Rüde,
 * "Analysis and comparison of boundary condition variants in the free-surface
 * lattice Boltzmann method": lattice Boltzmann collision with Guo gravity forcing
 * and streaming (Sec. 2.1), fill level, mass exchange, cell conversion with excess
 * mass and reinitialisation, anti-bounce-back free-surface condition with gas,
 * volume and Laplace pressure, Parker-Youngs normals (Sec. 2.2), and the four
 * reconstruction variants NBRC, NBKC, OM and OM3 (Sec. 3).
 *
 * Conventions shared by every entry point
 *  - Grid: nx*ny*nz cells, x fastest: idx = x + nx*(y + ny*z). Walls are ghost
 *    layers just outside the domain (halfway bounce-back puts the wall on the face).
 *  - Host arrays passed in are borrowed for the duration of the call and copied;
 *    host arrays passed out must hold the stated number of elements.
 *  - Every call returns an int status (FSLBM_OK = 0, negative on error), never
 *    throws across the ABI and never exits the process. fslbm_last_error() gives
 *    a message for the last failing call on a context.
 *  - A context is not thread-safe; separate contexts may run concurrently on
 *    separate streams.
 *  - Populations are kept in device memory as the POST-collision state f* of
 *    the current step (structure of arrays, q planes of N values; in the
 *    in-place layout a value's plane and cell alternate with the step parity,
 *    see fslbm_params.layout); reported
 *    fields are the pre-collision moments rho = sum f*, u = (sum c f* - rho g/2)/rho,
 *    which equal the moments of the populations after streaming.
 */
#ifndef FSLBM_H
#define FSLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FSLBM_ABI_VERSION 2

typedef struct fslbm_ctx fslbm_ctx;

enum {
  FSLBM_OK = 0,
  FSLBM_EINVAL = -1,    /* bad argument or parameter, or initial state violating the closed layer */
  FSLBM_ENOMEM = -2,    /* device allocation failed, the caller's arena is too small, or
                           (in-place layout) the interface outgrew the stash (sticky) */
  FSLBM_EDEVICE = -3,   /* HIP runtime error (launch, copy, fault reported by the runtime) */
  FSLBM_EUNSTABLE = -4, /* NaN, rho <= 0 or |u| >= c_s seen on the device (sticky) */
  FSLBM_ESTATE = -5,    /* call not valid in the context's state (e.g. after a device error) */
  FSLBM_EBUDGET = -6    /* server: request larger than the memory budget */
};

/* Reconstruction variants, Sec. 3.1-3.4. */
enum { FSLBM_NBRC = 1, FSLBM_NBKC = 2, FSLBM_OM = 3, FSLBM_OM3 = 4 };
/* Cell types (Sec. 2.2: gas, interface, liquid) and obstacles (Sec. 2.1). */
enum { FSLBM_GAS = 0, FSLBM_INTERFACE = 1, FSLBM_LIQUID = 2, FSLBM_NOSLIP = 3, FSLBM_FREESLIP = 4 };
enum { FSLBM_SRT = 0, FSLBM_TRT = 1 };
/* Population storage: binary64; binary32; binary16 holding f_i - w_i (FP32 arithmetic). */
enum { FSLBM_F64 = 0, FSLBM_F32 = 1, FSLBM_F16S = 2 };
/* Domain faces. */
enum { FSLBM_PERIODIC = 0, FSLBM_WALL_NOSLIP = 1, FSLBM_WALL_FREESLIP = 2 };
/* Population layout: two grids (each step reads one and writes the other) or one
 * grid updated in place (AA pattern). */
enum { FSLBM_TWO_GRID = 0, FSLBM_AA = 1 };

typedef struct {
  uint32_t abi_version;  /* must equal FSLBM_ABI_VERSION */
  int32_t nx, ny, nz;    /* interior cells, each >= 1 */
  int32_t q;             /* 19 (D3Q19) or 27 (D3Q27) */
  int32_t collision;     /* FSLBM_SRT (Sec. 2.1) or FSLBM_TRT */
  int32_t storage;       /* FSLBM_F64, FSLBM_F32 or FSLBM_F16S */
  int32_t boundary[6];   /* faces -x,+x,-y,+y,-z,+z: FSLBM_PERIODIC or FSLBM_WALL_* */
  int32_t variant;       /* FSLBM_NBRC .. FSLBM_OM3 */
  int32_t thurey_flux;   /* 1: interface cells without liquid (gas) neighbours are forced to
                            empty (fill) through the mass flux, Sec. 2.2; 0: plain flux */
  int32_t bubble_model;  /* 0: constant volume pressure; 1: one enclosed bubble,
                            p^V(t) = p^V(0) V(0)/V(t), Sec. 2.2; 2: every connected
                            region of gas and interface cells is a bubble with its own
                            p^V, its amount p^V V kept (Boyle), added on coalescence
                            and shared by gas volume on segmentation (fslbm_bubbles) */
  double tau;            /* relaxation time, > 0.5 (nu = (tau - 1/2)/3) */
  double trt_lambda;     /* TRT magic parameter, used only for FSLBM_TRT */
  double gravity[3];     /* acceleration; force density F = rho g, not weighted by phi */
  double rho_gas;        /* gas density at zero surface tension, = 3 p^V(0) */
  double sigma;          /* surface tension (0 = off): rho^G = 3 (p^V + sigma kappa) */
  double eps_phi;        /* conversion threshold (the paper uses 1e-2) */
  double tie_delta;      /* |n.c_i| <= tie_delta*max|n_a| counts as n.c_i = 0; 0 -> 1e-9 */
  double smagorinsky;    /* Smagorinsky constant C_S (Sec. 2.1 turbulence model), 0 = off;
                            the local tau replaces tau (TRT keeps trt_lambda) */
  int32_t layout;        /* FSLBM_TWO_GRID, or FSLBM_AA: one population grid, updated in
                            place (not in the paper, which does not fix a layout). A step
                            from an even step count pulls from the neighbours and writes
                            each outgoing value into the slot its opposite came from; a
                            step from an odd count reads and writes the cell's own slots.
                            The interface cells' own post-collision populations, which
                            the free-surface condition and the mass exchange (Sec. 2.2)
                            need after neighbours have overwritten them, are kept in two
                            stash buffers of max(N/8, 2F, 1024) cells (F the largest
                            face nx*ny, ny*nz or nx*nz; at most N) with a per-cell
                            entry index; a domain whose interface outgrows them
                            fails (at creation, or the run stops) with
                            FSLBM_ENOMEM. fslbm_create refuses (FSLBM_EINVAL) walls and
                            obstacles for which pull streaming takes some population
                            twice (free-slip faces or obstacles meeting obstacles at
                            corners). Results are bitwise those of FSLBM_TWO_GRID. */
} fslbm_params;

typedef struct {
  double total_mass;      /* liquid_mass + interface_mass + lost_mass (FP64) */
  double liquid_mass;     /* sum over liquid cells of rho */
  double interface_mass;  /* sum over interface cells of m */
  double lost_mass;       /* excess mass of converted cells that had no interface neighbour */
  double bubble_volume;   /* sum over non-obstacle cells of (1 - phi) */
  double p_volume;        /* current volume pressure p^V */
  int64_t n_liquid, n_interface, n_gas, step;
} fslbm_mass_report;

/* Device bytes fslbm_create needs for these parameters (for a caller-owned arena).
 * Errors: FSLBM_EINVAL for NULL pointers or invalid parameters. */
int fslbm_workspace_bytes(const fslbm_params* p, size_t* bytes);

/* Creates a simulation (Sec. 2.2 statement of the problem: cell types, fill levels,
 * density and velocity; interface mass m = phi * rho).
 * type, phi, rho, ux, uy, uz: host arrays of N elements. Populations start at the
 * equilibrium feq(rho, u) and are collided once, so the stored state is post-collision.
 * pdf_or_null: q*N host doubles of post-collision populations (as exported by
 *   fslbm_fields) for an exact resume; mass_or_null: N host doubles of interface mass
 *   (entries of other cells are ignored); phi then carries the fill levels of the
 *   saved state. The lost mass and the volume-pressure scalars start afresh (lost
 *   mass 0, p^V = p^V(0) = rho_gas/3, V(0) = the current gas volume) until
 *   fslbm_set_scalars restores them.
 * device_arena_or_null: caller-owned device memory of at least fslbm_workspace_bytes,
 *   kept alive until fslbm_destroy; NULL lets the library allocate (and free) it.
 * hip_stream: the hipStream_t all work is enqueued on (NULL = default stream).
 * Errors: FSLBM_EINVAL (bad parameters, liquid cell next to gas, unknown type),
 *   FSLBM_ENOMEM, FSLBM_EDEVICE. On error *out is NULL. */
int fslbm_create(const fslbm_params* p, const uint8_t* type, const double* phi, const double* rho,
                 const double* ux, const double* uy, const double* uz, const double* pdf_or_null,
                 const double* mass_or_null, void* device_arena_or_null, size_t arena_bytes,
                 void* hip_stream, fslbm_ctx** out);

/* Selects the reconstruction variant (Sec. 3) from the next step on.
 * Errors: FSLBM_EINVAL for an unknown variant or NULL context. */
int fslbm_set_variant(fslbm_ctx* ctx, int variant);

/* Enqueues nsteps time steps on the context's stream and returns without waiting.
 * Each step: stream + boundary condition + mass exchange + fill level + marks +
 * collision, then conversion, reinitialisation and excess-mass redistribution.
 * Errors: FSLBM_EINVAL (nsteps < 0), FSLBM_ESTATE (earlier device error), FSLBM_EDEVICE. */
int fslbm_step(fslbm_ctx* ctx, int64_t nsteps);

/* Waits for the stream and reports mass, counts and the bubble state (FP64,
 * deterministic reduction order). Returns FSLBM_EUNSTABLE if an instability was
 * detected since creation (the report is still filled). */
int fslbm_mass(fslbm_ctx* ctx, fslbm_mass_report* out);

/* For callers that cannot allocate or wait (code under HIP graph capture,
 * tight serving loops): the reduction of fslbm_mass, enqueued on the
 * context's stream without waiting, its per-block partial sums held in a
 * static device buffer of the library instead of the context's memory, and
 * its result written to device memory. Allocates nothing and calls no
 * allocating routine on success.
 * out_device: 8 doubles of device memory (caller-owned): total mass, liquid
 *   mass, interface mass, lost mass, bubble volume, n_liquid, n_interface,
 *   n_gas (counts as doubles); the same values, summed in the same order, as
 *   fslbm_mass reports for the same state. Valid once the stream reaches the
 *   call.
 * Limit: domains of at most 134217728 cells (16384 blocks of 8192 cells; the
 *   static buffer is 16384 * 7 doubles = 896 KiB per GPU, held until the
 *   process ends); larger ones get FSLBM_EINVAL and a message (use fslbm_mass).
 * The static buffer is shared by every context on one GPU: calls that may
 *   overlap on one GPU (different streams, different host threads) race;
 *   calls ordered on one stream do not. No status check: an instability is
 *   reported by the next fslbm_mass or fslbm_fields.
 * Errors: FSLBM_EINVAL (NULL, domain too large), FSLBM_ESTATE, FSLBM_EDEVICE. */
int fslbm_mass_noalloc(fslbm_ctx* ctx, double* out_device);

/* Waits for the stream and copies fields out (any pointer may be NULL):
 * type (N bytes), phi, rho, ux, uy, uz, mass (N doubles each; mass is m for
 * interface cells, rho for liquid cells, 0 for gas), pdf (q*N doubles,
 * post-collision populations, gas cells 0). Returns FSLBM_EUNSTABLE like fslbm_mass. */
int fslbm_fields(fslbm_ctx* ctx, uint8_t* type, double* phi, double* rho, double* ux, double* uy,
                 double* uz, double* mass, double* pdf);

/* Number of interface cells in the compacted interface list and, if list is not
 * NULL, the list itself (ascending cell indices, at most max entries). Syncs. */
int fslbm_interface_list(fslbm_ctx* ctx, int32_t* list, int64_t max, int64_t* count);

/* Tracked bubbles (bubble_model 2: Sec. 2.2 volume-pressure equation, each
 * connected region of gas and interface cells its own bubble, followed
 * through coalescence and segmentation). Waits for the stream; *count = the
 * number of bubbles (0 for the other models) and, for the first max of them
 * in ascending label order, label[i] = the bubble's smallest cell index,
 * volume[i] = sum of 1 - phi over its cells, pressure[i] = its volume
 * pressure p^V. Arrays are host memory owned by the caller (may be NULL when
 * max is 0). Errors: FSLBM_EINVAL (NULL count, or NULL arrays with max > 0);
 * FSLBM_EDEVICE if the labelling did not complete; FSLBM_EUNSTABLE as for
 * fslbm_mass (the arrays are still filled). */
int fslbm_bubbles(fslbm_ctx* ctx, int64_t* label, double* volume, double* pressure, int64_t max,
                  int64_t* count);

/* Kernel timing for measurement. fslbm_set_timing(ctx, capacity) with
 * capacity > 0 brackets the next `capacity` launches of the streaming kernel
 * (pull streaming, free-surface condition, mass exchange and collision of
 * every liquid and interface cell) with HIP events on the context's stream (capacity 0
 * turns timing off and releases the events). fslbm_kernel_time syncs and
 * returns the number of timed launches and their summed duration in ms.
 * Errors: FSLBM_EINVAL (NULL, capacity < 0), FSLBM_EDEVICE. */
int fslbm_set_timing(fslbm_ctx* ctx, int64_t capacity);
int fslbm_kernel_time(fslbm_ctx* ctx, int64_t* launches, double* total_ms);

/* Step launches: with enable = 1 (the default) fslbm_step replays captured
 * HIP graphs of 8 steps, then of 2 steps, when the context's stream is not the
 * NULL stream and timing is off (an odd last step is launched kernel by
 * kernel); enable = 0 always launches kernel by kernel. Results are identical
 * either way. There is one graph per length and step parity; each is captured
 * on first use, or all four at once by fslbm_set_graphs(ctx, 1) (capture
 * records the launches without running them), so that timed steps need not
 * include it. Errors: FSLBM_EINVAL (NULL), FSLBM_ESTATE, FSLBM_EDEVICE
 * (capture failed). */
int fslbm_set_graphs(fslbm_ctx* ctx, int enable);

/* Compaction tile size: every thread of a 1024-thread compaction tile scans
 * cells_per_thread consecutive cells (16 times a power of two). The library
 * picks the smallest size that keeps the tile count within its status array;
 * a larger one (fewer, longer tiles) is accepted, a smaller one is not. It
 * changes the work split only: results are identical. For tuning and for
 * exercising every tile shape on small domains. Errors: FSLBM_EINVAL (NULL,
 * not 16 times a power of two, below the library's size, above 4096). */
int fslbm_set_compaction_tile(fslbm_ctx* ctx, int cells_per_thread);

/* Scalars of a run's state beside its fields (Sec. 2.2): out/in[0] = lost
 * mass (excess mass of converted cells that had no interface neighbour,
 * counted in the total mass), [1] = the volume pressure p^V, [2] = p^V(0),
 * [3] = V(0) of the volume-pressure equation p^V = p^V(0) V(0)/V. Together with
 * fslbm_fields (type, phi, mass, pdf) they are the state an exact resume needs:
 * fslbm_create(pdf, mass) followed by fslbm_set_scalars continues a run with
 * constant pressure or one bubble (bubble_model 0 or 1) as if uninterrupted;
 * with tracked bubbles (bubble_model 2) the bubbles restart at p^V(0).
 * fslbm_get_scalars waits for the stream; fslbm_set_scalars takes effect for
 * the next step and waits for the stream. in/out are 4 host doubles.
 * Errors: FSLBM_EINVAL (NULL, non-finite values, V(0) <= 0 with bubble_model 1),
 * FSLBM_ESTATE, FSLBM_EDEVICE. */
int fslbm_get_scalars(fslbm_ctx* ctx, double out[4]);
int fslbm_set_scalars(fslbm_ctx* ctx, const double in[4]);

/* Releases the context (NULL-safe; never fails). Does not free a caller arena. */
void fslbm_destroy(fslbm_ctx* ctx);

/* Static message for a status code. */
const char* fslbm_strerror(int status);
/* Message for the last failing call on ctx (or the last fslbm_create failure
 * when ctx is NULL). The pointer stays valid until the next call on ctx. */
const char* fslbm_last_error(const fslbm_ctx* ctx);

/* ------------------------------------------------------------------------
 * Serving: many independent runs batched on one GPU.
 *
 * A server owns one device pool of hbm_budget_bytes (allocated at create) and
 * up to max_slots resident runs. Submitted runs wait in a FIFO queue and are
 * admitted, in order, while a slot is free and the pool has room for their
 * workspace (fslbm_workspace_bytes); a run that can never fit is rejected at
 * submit. Every resident run keeps its whole state in its part of the pool;
 * each step phase is one launch covering all resident runs of the same
 * population format, lattice and collision (one block range per run), so
 * runs of different sizes, variants and parameters advance together. A run
 * leaves when it has taken its steps: its mass report and fill levels are kept
 * for fslbm_server_result, its memory and slot go to the next queued run.
 * A run's results do not depend on which other runs share the launches (each
 * run's cells are computed by the same code as in a single context).
 * Runs with surface tension (sigma > 0) add a smoothing and a curvature
 * launch before the step, runs with one enclosed bubble (bubble_model 1) a
 * volume and a volume-pressure launch after it, each covering the runs of the
 * group that need it, and runs with tracked bubbles (bubble_model 2) the
 * seven bubble passes after it (Sec. 2.2 volume-pressure equation for every
 * bubble), again only over those runs. The server is not thread-safe.
 * ------------------------------------------------------------------------ */
typedef struct fslbm_server fslbm_server;

typedef struct {
  int64_t queued, resident, completed, ticks;
  uint64_t bytes_in_use, peak_bytes_in_use, budget_bytes;
} fslbm_server_stats;

/* hbm_budget_bytes: device pool size (hipMalloc'ed once); max_slots: resident
 * runs at most (1..4096); hip_stream: stream of all server work (borrowed,
 * NULL = default stream). Errors: FSLBM_EINVAL, FSLBM_ENOMEM. */
int fslbm_server_create(size_t hbm_budget_bytes, int max_slots, void* hip_stream, fslbm_server** out);

/* Queues one run of nsteps steps (> 0) from the given initial fields (the
 * arrays of fslbm_create, copied: the caller may free them on return).
 * req_id receives the run's id (increasing from 1). Errors: FSLBM_EINVAL
 * (parameters, nsteps <= 0, workspace above the budget),
 * FSLBM_ENOMEM (host memory). */
int fslbm_server_submit(fslbm_server* srv, const fslbm_params* p, const uint8_t* type,
                        const double* phi, const double* rho, const double* ux, const double* uy,
                        const double* uz, int64_t nsteps, uint64_t* req_id);

/* Runs up to `ticks` batched steps (a tick advances every resident run by one
 * step), retiring finished runs and admitting queued ones between ticks as
 * slots and pool memory free up; returns early when nothing is resident or
 * queued. Waits for the device only where a run finishes. Launch groups
 * (runs sharing storage, lattice, collision and addressing) run side by side
 * on streams the server owns, ordered after and before the server's stream
 * by events, so work the caller queues on that stream still follows the
 * ticks. Errors: FSLBM_EDEVICE (the server is unusable afterwards). */
int fslbm_server_advance(fslbm_server* srv, int64_t ticks);

/* Ids and statuses (FSLBM_OK, or FSLBM_EUNSTABLE for a run that became
 * unstable) of runs finished since the last poll, at most max; n_done
 * receives the number written. */
int fslbm_server_poll(fslbm_server* srv, uint64_t* done_ids, int* statuses, int max, int* n_done);

/* Mass report and, if phi_out is not NULL, the N fill levels of a finished
 * run; releases the stored result. Errors: FSLBM_EINVAL (unknown or not yet
 * finished id). */
int fslbm_server_result(fslbm_server* srv, uint64_t req_id, fslbm_mass_report* report,
                        double* phi_out);

/* Counters of the server (queue length, resident runs, pool use). */
int fslbm_server_stats_get(const fslbm_server* srv, fslbm_server_stats* out);

/* Releases every run and the pool (NULL-safe). */
void fslbm_server_destroy(fslbm_server* srv);

#ifdef __cplusplus
}
#endif
#endif
