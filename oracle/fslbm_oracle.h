/*
 * Plain FP64 CPU oracle of one free-surface lattice Boltzmann (FSLBM) time step.
 *
 * TEST INFRASTRUCTURE ONLY. This library is the slow, obviously-correct
 * definition the GPU library is checked against. Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never does. It shares no code, header, table or constant with
 * the HIP library: the lattice tables below are written out independently.
 *
 * What it computes (Schwarzmeier & Rüde, "Analysis and comparison of boundary
 * condition variants in the free-surface lattice Boltzmann method"):
 *   Sec. 2.1  collision (SRT, plus a TRT variant), equilibrium, moments, Guo
 *             forcing, bounce-back / specular walls;
 *   Sec. 2.2  fill level, mass, mass flux, conversion thresholds, excess mass,
 *             reinitialisation, anti-bounce-back free-surface condition, gas /
 *             volume / Laplace pressure, Parker-Youngs normal, curvature;
 *   Sec. 3    the four reconstruction variants NBRC, NBKC, OM, OM3.
 * The order of the sub-steps inside one time step is not stated in the paper;
 * the canonical order used here is documented step by step in fslbm_oracle.c.
 *
 * Storage convention: the state between steps is the PRE-collision population
 * f (x fastest: idx = x + nx*(y + ny*z); f[i*N + idx]). Fields reported after
 * a step are pre-collision moments rho = sum f, u = (sum c f + rho g / 2)/rho.
 */
#ifndef FSLBM_ORACLE_H
#define FSLBM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_GAS = 0, ORC_INTERFACE = 1, ORC_LIQUID = 2, ORC_NOSLIP = 3, ORC_FREESLIP = 4 };
enum { ORC_PERIODIC = 0, ORC_WALL_NOSLIP = 1, ORC_WALL_FREESLIP = 2 };
enum { ORC_NBRC = 1, ORC_NBKC = 2, ORC_OM = 3, ORC_OM3 = 4 };
enum { ORC_SRT = 0, ORC_TRT = 1 };
enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_EUNSTABLE = -4 };

typedef struct {
  int32_t nx, ny, nz;
  int32_t q;             /* 19 or 27 */
  int32_t collision;     /* ORC_SRT / ORC_TRT */
  int32_t boundary[6];   /* faces -x,+x,-y,+y,-z,+z */
  int32_t variant;       /* ORC_NBRC..ORC_OM3 */
  int32_t thurey_flux;   /* 1: forced fill/empty flux modification */
  int32_t bubble_model;  /* 0: constant volume pressure, 1: one enclosed bubble,
                            2: every bubble tracked (coalescence, segmentation) */
  double tau, trt_lambda;
  double gravity[3];
  double rho_gas;        /* gas density at zero surface tension (= 3 p^V) */
  double sigma;          /* surface tension, 0 = off */
  double eps_phi;        /* conversion threshold */
  double tie_delta;      /* band for n.c = 0 decisions, relative to max|n_a| */
  double smagorinsky;    /* Smagorinsky constant C_S of the LES model (0 = off) */
} orc_params;

typedef struct orc_sim orc_sim;

/* Builds a simulation from initial cell types, fill levels, densities and
 * equilibrium velocities (all N-arrays, borrowed). Interface mass is phi*rho.
 * Returns ORC_EINVAL for bad parameters or a liquid cell touching gas. */
int orc_create(const orc_params* p, const uint8_t* type, const double* phi,
               const double* rho, const double* ux, const double* uy,
               const double* uz, orc_sim** out);
void orc_destroy(orc_sim* s);

/* Advances n steps; returns ORC_EUNSTABLE (sticky) on NaN, rho <= 0, |u| >= c_s. */
int orc_step(orc_sim* s, int64_t n);
int orc_set_variant(orc_sim* s, int variant);

/* Pre-collision fields at the current step; any pointer may be NULL.
 * pdf: q*N pre-collision populations (gas cells 0). */
void orc_fields(const orc_sim* s, uint8_t* type, double* phi, double* rho,
                double* ux, double* uy, double* uz, double* mass, double* pdf);
/* Post-collision populations f* = collide(f) of the current state (q*N),
 * gas cells 0. This is what a stream-collide-fused code stores. */
void orc_post_collision(const orc_sim* s, double* pdf_star);

typedef struct {
  double total_mass, liquid_mass, interface_mass, lost_mass, bubble_volume, p_volume;
  int64_t n_liquid, n_interface, n_gas, step;
} orc_report;
void orc_mass(const orc_sim* s, orc_report* r);
/* Tracked bubbles (bubble_model 2), ascending by label (the smallest cell
 * index of the bubble): label, gas volume and volume pressure of the first
 * `cap` of them. Returns the number of bubbles (0 for other models). */
int64_t orc_bubbles(const orc_sim* s, int64_t* label, double* volume, double* pressure, int64_t cap);

/* Threads of the per-cell loops (default: one below 65536 cells, OpenMP's
 * maximum above). The result is
 * bitwise the same for every thread count. */
int orc_set_threads(orc_sim* s, int threads);

/* The state between steps, copied verbatim (no arithmetic): cell types,
 * pre-collision populations (q*N), the mass array (interface cells: m; other
 * cells hold 0), fill levels of every cell, and the scalars
 * {lost mass, p^V, p^V(0), V(0)}. Any pointer may be NULL. */
void orc_export_state(const orc_sim* s, uint8_t* type, double* pdf, double* mass, double* phi,
                      double scalars[4]);
/* Replaces the state by one of the same shape, verbatim; the next step is
 * number `step`. Tracked bubbles (bubble_model 2) are labelled afresh from the
 * imported types, every bubble starting at p^V(0). */
int orc_import_state(orc_sim* s, const uint8_t* type, const double* pdf, const double* mass,
                     const double* phi, const double scalars[4], int64_t step);

/* Isolated routines exposed for the pins. */
/* Equilibrium of the given lattice (q = 19/27); feq has q entries. */
void orc_equilibrium(int q, double rho, const double u[3], double* feq);
/* Lattice velocity c_i (3 ints) and weight. */
void orc_lattice(int q, int i, int c[3], double* w);
int orc_opposite(int q, int i);
/* One collision of a single cell: f (q) -> fs (q); returns collision velocity in u
 * and, if tau_out is not NULL, the relaxation time used (tau, or tau0 + tau_t
 * with the Smagorinsky model when cs > 0). */
void orc_collide_cell(int q, int collision, double tau, double lambda, double cs, const double g[3],
                      const double* f, double* fs, double u[3], double* tau_out);
/* Reconstruction set of one interface cell: given the normal n, the gas-source
 * mask (bit i set when x - c_i is gas) and the variant, writes R[i] = 1 for
 * every direction overwritten by the anti-bounce-back condition (forced gas
 * sources included). */
void orc_reconstruct_set(int q, int variant, const double n[3], uint32_t gas_src_mask,
                         double tie_delta, uint8_t* R);
/* Anti-bounce-back value for direction i: 2 feq+_i(rho_g, u) - fs_ibar. */
double orc_bc_value(int q, int i, double rho_g, const double u[3], double fs_ibar);
/* Parker-Youngs normal of cell (x,y,z) from the current fill levels. */
void orc_normal(const orc_sim* s, int x, int y, int z, double n[3]);
/* Curvature kappa = -div(n_hat) from the K8-smoothed fill level (interface cells). */
double orc_curvature(const orc_sim* s, int x, int y, int z);
/* Mass-flux classes (0 std, 1 no liquid nb, 2 no gas nb) of an interface cell. */
int orc_thurey_class(const orc_sim* s, int x, int y, int z);

#ifdef __cplusplus
}
#endif
#endif
