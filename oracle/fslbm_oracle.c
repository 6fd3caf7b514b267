/*
 * Plain FP64 CPU oracle of the free-surface lattice Boltzmann time step.
 *
 * TEST INFRASTRUCTURE ONLY (see fslbm_oracle.h). Written for readability:
 * every sub-step is a separate loop over all cells in index order, every sum
 * runs over the direction index in ascending order, no blocking, no fusion.
 * Build with -O2 -ffp-contract=off and without fast-math so that each
 * operation is one correctly rounded IEEE-754 binary64 operation.
 *
 * Threads: loops in which every iteration writes only its own cell are
 * spread over OpenMP threads (the iterations are independent, so the result
 * is bitwise the same for any thread count); every sum over cells (lost
 * mass, bubble volumes and amounts, mass reports) stays a serial loop in
 * index order.
 *
 * Parity status: every function below is pinned by a CPU test against a
 * closed form, an invariant or a brute-force enumeration. The readings of
 * what the paper delegates to cited work (the forced fill/empty flux table,
 * the near-obstacle normal, the reinitialisation averages, the lost-mass
 * fallback, the K8 smoothing next to obstacles, the free-slip edge rules)
 * are pinned by consequences of their stated intent: a cell that should
 * empty only gives mass, one that should fill only receives; a new cell
 * carries the equilibrium of the mean of exactly its allowed neighbours after
 * streaming; unplaceable excess mass is booked exactly; a flat surface keeps
 * its normal and zero curvature up to walls; free-slip faces and edges keep
 * the tangential momentum. The exact tables of the cited works are not
 * available, so another reading consistent with the same intent would not be
 * told apart. The tracked-bubble rules (also delegated) are pinned by
 * invariants: connected components, Boyle's law per bubble, amounts added on
 * coalescence, pressure kept on segmentation.
 */
#include "fslbm_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------------
 * Lattice (Sec. 2.1: DdQq velocity sets; weights are the standard ones).
 * Direction order: rest, 6 faces, 12 edges, 8 corners; D3Q19 is the first 19.
 * Opposite of i > 0: odd i -> i + 1, even i -> i - 1.
 * ------------------------------------------------------------------------- */
static const int CV[27][3] = {
    {0, 0, 0},
    {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},   {0, -1, 0},  {0, 0, 1},   {0, 0, -1},
    {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},  {-1, 1, 0},
    {1, 0, 1},   {-1, 0, -1}, {1, 0, -1},  {-1, 0, 1},
    {0, 1, 1},   {0, -1, -1}, {0, 1, -1},  {0, -1, 1},
    {1, 1, 1},   {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},
    {1, -1, 1},  {-1, 1, -1}, {-1, 1, 1},  {1, -1, -1}};

static double weight(int q, int i) {
  int n2 = CV[i][0] * CV[i][0] + CV[i][1] * CV[i][1] + CV[i][2] * CV[i][2];
  if (q == 19) {
    if (n2 == 0) return 1.0 / 3.0;
    if (n2 == 1) return 1.0 / 18.0;
    return 1.0 / 36.0;
  }
  if (n2 == 0) return 8.0 / 27.0;
  if (n2 == 1) return 2.0 / 27.0;
  if (n2 == 2) return 1.0 / 54.0;
  return 1.0 / 216.0;
}

int orc_opposite(int q, int i) {
  (void)q;
  if (i == 0) return 0;
  return (i & 1) ? i + 1 : i - 1;
}

void orc_lattice(int q, int i, int c[3], double* w) {
  c[0] = CV[i][0];
  c[1] = CV[i][1];
  c[2] = CV[i][2];
  *w = weight(q, i);
}

static int dir_index(int q, int cx, int cy, int cz) {
  for (int i = 0; i < q; ++i)
    if (CV[i][0] == cx && CV[i][1] == cy && CV[i][2] == cz) return i;
  return -1;
}

/* ---------------------------------------------------------------------------
 * Simulation state.
 * ------------------------------------------------------------------------- */
struct orc_sim {
  orc_params p;
  int q;
  long N;
  uint8_t* type;
  double* f;      /* pre-collision populations, q*N */
  double* fs;     /* post-collision populations of the current step, q*N */
  double* fn;     /* populations after streaming + boundary condition, q*N */
  double* m;      /* liquid mass of interface cells */
  double* phi;    /* fill level of every cell (liquid 1, gas 0) */
  double* ut;     /* collision velocity, 3*N */
  double* rhoG;   /* gas density per interface cell */
  double* rhon;   /* density after streaming */
  double* phis;   /* K8-smoothed fill level (surface tension only) */
  double* share;  /* excess-mass share handed out by a converted cell */
  uint8_t* mark;  /* 0 none, 1 to liquid, 2 to gas */
  uint8_t* conv;  /* conversion of this step, see CONV_* */
  uint8_t* cls;   /* flux class of interface cells */
  uint8_t* ntype; /* type after conversion */
  double m_lost;
  double pV, pV0, V0;
  /* tracked bubbles (bubble_model 2): label per cell (-1: no bubble), and at
   * each bubble's label index its gas amount and pressure; per cell the
   * volume pressure of its bubble; work arrays of the update */
  int32_t *blab, *bnew, *btgt;
  double *bamt, *bpr, *bpc, *bV, *bW, *bR, *bnn;
  uint8_t* bhas;
  long* bqueue;
  int64_t step;
  int status;
  int threads; /* OpenMP threads of the per-cell loops */
};

enum { MARK_NONE = 0, MARK_L = 1, MARK_G = 2 };
enum { CONV_NONE = 0, CONV_TO_LIQ = 1, CONV_TO_GAS = 2, CONV_NEW_FROM_GAS = 3, CONV_NEW_FROM_LIQ = 4 };
enum { CLS_STD = 0, CLS_NOLIQ = 1, CLS_NOGAS = 2 };

static int is_obstacle(int t) { return t == ORC_NOSLIP || t == ORC_FREESLIP; }
static int is_fluid(int t) { return t == ORC_LIQUID || t == ORC_INTERFACE; }

/* Type of the cell at (x,y,z) + (dx,dy,dz). A periodic face wraps the
 * coordinate; a coordinate beyond a wall face gives that wall's obstacle type
 * (walls are ghost layers just outside the domain, so a halfway bounce-back
 * puts the wall on the domain face). Where a no-slip and a free-slip face are
 * both crossed (an edge or corner ghost), no-slip wins. *idx is the wrapped
 * index, or -1 for a ghost. */
static int lookup(const orc_sim* s, int x, int y, int z, int dx, int dy, int dz, long* idx) {
  int c[3] = {x + dx, y + dy, z + dz};
  const int n[3] = {s->p.nx, s->p.ny, s->p.nz};
  int wall = 0;
  for (int a = 0; a < 3; ++a) {
    int face;
    if (c[a] < 0)
      face = 2 * a;
    else if (c[a] >= n[a])
      face = 2 * a + 1;
    else
      continue;
    if (s->p.boundary[face] == ORC_PERIODIC) {
      c[a] = ((c[a] % n[a]) + n[a]) % n[a];
    } else {
      int wt = s->p.boundary[face] == ORC_WALL_NOSLIP ? ORC_NOSLIP : ORC_FREESLIP;
      if (wall != ORC_NOSLIP) wall = wt;
    }
  }
  if (wall) {
    *idx = -1;
    return wall;
  }
  *idx = c[0] + (long)s->p.nx * (c[1] + (long)s->p.ny * c[2]);
  return s->type[*idx];
}

static void coords(const orc_sim* s, long idx, int* x, int* y, int* z) {
  *x = (int)(idx % s->p.nx);
  *y = (int)((idx / s->p.nx) % s->p.ny);
  *z = (int)(idx / ((long)s->p.nx * s->p.ny));
}

/* ---------------------------------------------------------------------------
 * Sec. 2.1: equilibrium (second order in u, c_s^2 = 1/3).
 * ------------------------------------------------------------------------- */
void orc_equilibrium(int q, double rho, const double u[3], double* feq) {
  double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < q; ++i) {
    double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
    feq[i] = weight(q, i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
  }
}

/* Moments, Sec. 2.1: rho = sum f; u = (sum c f + F/2) / rho with F = rho g
 * (the gravitational force density, not weighted by the fill level, Sec. 2.2). */
static void moments(int q, const double* f, long stride, const double g[3], double* rho_out,
                    double u[3]) {
  double rho = 0.0, j0 = 0.0, j1 = 0.0, j2 = 0.0;
  for (int i = 0; i < q; ++i) rho += f[i * stride];
  for (int i = 0; i < q; ++i) {
    double fi = f[i * stride];
    j0 += CV[i][0] * fi;
    j1 += CV[i][1] * fi;
    j2 += CV[i][2] * fi;
  }
  u[0] = (j0 + 0.5 * (rho * g[0])) / rho;
  u[1] = (j1 + 0.5 * (rho * g[1])) / rho;
  u[2] = (j2 + 0.5 * (rho * g[2])) / rho;
  *rho_out = rho;
}

/* Smagorinsky model (Sec. 2.1, turbulence relaxation time): momentum fluxes
 * of the non-equilibrium part Q_ab = sum_i c_ia c_ib (f_i - feq_i), filtered
 * flux Qbar = sqrt(2 sum_ab Q_ab Q_ab), and the total relaxation time
 * tau = tau0 + tau_t with tau_t = (sqrt(tau0^2 + 2 sqrt(2) C_S^2 Qbar /
 * (rho c_s^4)) - tau0) / 2 (filter width 1). The printed expression drops the
 * parentheses around the difference, which would give tau = tau0/2 at
 * Qbar = 0; the parenthesised form is the one that reduces to tau0. */
static double les_tau(int q, double tau0, double cs, double rho, const double* f,
                      const double* feq) {
  double Qab[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int i = 0; i < q; ++i) Qab[a][b] += CV[i][a] * CV[i][b] * (f[i] - feq[i]);
  double s2 = 0.0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) s2 += Qab[a][b] * Qab[a][b];
  double Qbar = sqrt(2.0 * s2);
  double cs4 = 1.0 / 9.0;
  double tau_t = 0.5 * (sqrt(tau0 * tau0 + 2.0 * sqrt(2.0) * cs * cs * Qbar / (rho * cs4)) - tau0);
  return tau0 + tau_t;
}

/* Collision of one cell, Sec. 2.1: f* = f - omega (f - feq) + (1 - omega/2) S
 * with the Guo source S_i = w_i [3 (c_i - u).F + 9 (c_i.u)(c_i.F)].
 * The relaxation term is subtracted (standard BGK; the printed operator has
 * the opposite sign). TRT (not in the paper): the same step applied to the
 * symmetric (+) and antisymmetric (-) parts with rates omega+ = 1/tau and
 * 1/omega- = 1/2 + lambda/(tau - 1/2); lambda = (tau - 1/2)^2 reduces it to SRT.
 * With cs > 0, tau is the Smagorinsky total relaxation time of this cell. */
void orc_collide_cell(int q, int collision, double tau, double lambda, double cs, const double g[3],
                      const double* f, double* fs, double u[3], double* tau_out) {
  double rho;
  moments(q, f, 1, g, &rho, u);
  double F[3] = {rho * g[0], rho * g[1], rho * g[2]};
  double feq[27], S[27];
  double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < q; ++i) {
    double w = weight(q, i);
    double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
    double cF = CV[i][0] * F[0] + CV[i][1] * F[1] + CV[i][2] * F[2];
    double cmuF = (CV[i][0] - u[0]) * F[0] + (CV[i][1] - u[1]) * F[1] + (CV[i][2] - u[2]) * F[2];
    feq[i] = w * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
    S[i] = w * (3.0 * cmuF + 9.0 * cu * cF);
  }
  if (cs > 0.0) tau = les_tau(q, tau, cs, rho, f, feq);
  if (tau_out) *tau_out = tau;
  double omega = 1.0 / tau;
  if (collision == ORC_SRT) {
    for (int i = 0; i < q; ++i)
      fs[i] = f[i] - omega * (f[i] - feq[i]) + (1.0 - 0.5 * omega) * S[i];
    return;
  }
  double omega_m = 1.0 / (0.5 + lambda / (tau - 0.5));
  for (int i = 0; i < q; ++i) {
    int ib = orc_opposite(q, i);
    double fp = 0.5 * (f[i] + f[ib]), fm = 0.5 * (f[i] - f[ib]);
    double ep = 0.5 * (feq[i] + feq[ib]), em = 0.5 * (feq[i] - feq[ib]);
    double sp = 0.5 * (S[i] + S[ib]), sm = 0.5 * (S[i] - S[ib]);
    fs[i] = f[i] - omega * (fp - ep) - omega_m * (fm - em) + (1.0 - 0.5 * omega) * sp +
            (1.0 - 0.5 * omega_m) * sm;
  }
}

/* ---------------------------------------------------------------------------
 * Sec. 2.2, anti-bounce-back condition: f_i(x) = feq_i(rhoG,u) + feq_ibar(rhoG,u)
 * - f*_ibar(x). The odd terms cancel, leaving 2 feq+_i - f*_ibar.
 * ------------------------------------------------------------------------- */
double orc_bc_value(int q, int i, double rho_g, const double u[3], double fs_ibar) {
  double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
  return 2.0 * weight(q, i) * rho_g * (1.0 + 4.5 * cu * cu - 1.5 * usq) - fs_ibar;
}

/* Sec. 3: reconstruction sets. Directions whose source is gas are always
 * reconstructed (Sec. 2.2: they are missing). On top of that:
 *   NBRC (Sec. 3.1): every i with n.c_i >= 0, the rest direction included;
 *   NBKC (Sec. 3.2): every i != 0 with n.c_i >= 0 (directions perpendicular to
 *         n are reconstructed, only the rest population is kept);
 *   OM   (Sec. 3.3): nothing else;
 *   OM3  (Sec. 3.4): if fewer than three are missing, the NBKC set (the text
 *         names NBKC as the fallback used in the study).
 * n.c_i counts as zero when |n.c_i| <= delta * max_a |n_a|; n = 0 makes every
 * product zero. */
void orc_reconstruct_set(int q, int variant, const double n[3], uint32_t gas_src_mask,
                         double tie_delta, uint8_t* R) {
  double nmax = fabs(n[0]);
  if (fabs(n[1]) > nmax) nmax = fabs(n[1]);
  if (fabs(n[2]) > nmax) nmax = fabs(n[2]);
  int missing = 0;
  for (int i = 0; i < q; ++i) {
    R[i] = (uint8_t)((gas_src_mask >> i) & 1u);
    missing += R[i];
  }
  int add_normal = 0, with_rest = 0;
  if (variant == ORC_NBRC) {
    add_normal = 1;
    with_rest = 1;
  } else if (variant == ORC_NBKC) {
    add_normal = 1;
  } else if (variant == ORC_OM3 && missing < 3) {
    add_normal = 1;
  }
  if (!add_normal) return;
  for (int i = (with_rest ? 0 : 1); i < q; ++i) {
    double dot = n[0] * CV[i][0] + n[1] * CV[i][1] + n[2] * CV[i][2];
    if (dot >= -tie_delta * nmax) R[i] = 1;
  }
}

/* Sec. 2.2, interface normal n = grad(phi) by the Parker-Youngs weighted
 * central difference over the 3x3x3 neighbourhood: for axis a,
 * n_a = sum_{b,c in -1..1} W_b W_c [phi(x + e_a + b e_a' + c e_a'') -
 * phi(x - e_a + b e_a' + c e_a'')] with W_0 = 2, W_+-1 = 1.
 * Near obstacles the stencil must not read obstacle cells: an obstacle point
 * takes the fill level of the centre cell (a reading; pinned by a flat surface
 * meeting walls keeping its normal exactly along them). */
static void normal_of(const orc_sim* s, const double* fld, int x, int y, int z, double n[3]) {
  static const double W[3] = {1.0, 2.0, 1.0};
  long i0 = x + (long)s->p.nx * (y + (long)s->p.ny * z);
  double v0 = fld[i0];
  for (int a = 0; a < 3; ++a) {
    int a1 = (a + 1) % 3, a2 = (a + 2) % 3;
    double sum = 0.0;
    for (int b = -1; b <= 1; ++b) {
      for (int c = -1; c <= 1; ++c) {
        int dp[3] = {0, 0, 0}, dm[3] = {0, 0, 0};
        dp[a] = 1;
        dm[a] = -1;
        dp[a1] = dm[a1] = b;
        dp[a2] = dm[a2] = c;
        long ip, im;
        int tp = lookup(s, x, y, z, dp[0], dp[1], dp[2], &ip);
        int tm = lookup(s, x, y, z, dm[0], dm[1], dm[2], &im);
        double vp = is_obstacle(tp) ? v0 : fld[ip];
        double vm = is_obstacle(tm) ? v0 : fld[im];
        sum += W[b + 1] * W[c + 1] * (vp - vm);
      }
    }
    n[a] = sum;
  }
}

void orc_normal(const orc_sim* s, int x, int y, int z, double n[3]) {
  normal_of(s, s->phi, x, y, z, n);
}

/* Smoothing of the fill level with the K8 kernel K(r) = (1 - r^2/h^2)^4,
 * support radius h = 2 (Sec. 2.2); with unit spacing only offsets with
 * r^2 < 4, i.e. the 3x3x3 box, carry weight. Obstacle cells are left out and
 * the weights renormalised over the rest (a reading; pinned by a flat surface
 * keeping zero curvature next to walls). */
static double smooth_phi(const orc_sim* s, int x, int y, int z) {
  double num = 0.0, den = 0.0;
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        long j;
        int t = lookup(s, x, y, z, dx, dy, dz, &j);
        if (is_obstacle(t)) continue;
        double r2 = (double)(dx * dx + dy * dy + dz * dz);
        double b = 1.0 - r2 / 4.0;
        double k = b * b * b * b;
        num += k * s->phi[j];
        den += k;
      }
  return num / den;
}

/* Unit normal from the smoothed fill level (zero where the gradient vanishes). */
static void unit_normal_smoothed(const orc_sim* s, int x, int y, int z, double nh[3]) {
  double n[3];
  normal_of(s, s->phis, x, y, z, n);
  double len = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  if (len > 0.0) {
    nh[0] = n[0] / len;
    nh[1] = n[1] / len;
    nh[2] = n[2] / len;
  } else {
    nh[0] = nh[1] = nh[2] = 0.0;
  }
}

/* Sec. 2.2, curvature kappa = -div(n_hat), central differences of the unit
 * normal of the smoothed fill level at the six face neighbours; an obstacle
 * neighbour contributes the centre's normal. Requires s->phis to be current. */
static double curvature_at(const orc_sim* s, int x, int y, int z) {
  double nc[3];
  unit_normal_smoothed(s, x, y, z, nc);
  double div = 0.0;
  for (int a = 0; a < 3; ++a) {
    int d[3] = {0, 0, 0};
    double np[3], nm[3];
    long j;
    d[a] = 1;
    int tp = lookup(s, x, y, z, d[0], d[1], d[2], &j);
    if (is_obstacle(tp)) {
      np[a] = nc[a];
    } else {
      int xx, yy, zz;
      coords(s, j, &xx, &yy, &zz);
      unit_normal_smoothed(s, xx, yy, zz, np);
    }
    d[a] = -1;
    int tm = lookup(s, x, y, z, d[0], d[1], d[2], &j);
    if (is_obstacle(tm)) {
      nm[a] = nc[a];
    } else {
      int xx, yy, zz;
      coords(s, j, &xx, &yy, &zz);
      unit_normal_smoothed(s, xx, yy, zz, nm);
    }
    div += 0.5 * (np[a] - nm[a]);
  }
  return -div;
}

static void update_smoothed(orc_sim* s) {
#pragma omp parallel for num_threads(s->threads) schedule(static)
  for (long c = 0; c < s->N; ++c) {
    int x, y, z;
    coords(s, c, &x, &y, &z);
    s->phis[c] = is_obstacle(s->type[c]) ? 0.0 : smooth_phi(s, x, y, z);
  }
}

double orc_curvature(const orc_sim* s, int x, int y, int z) {
  /* the smoothed field is refreshed by the caller-visible state: recompute */
  orc_sim* w = (orc_sim*)s;
  update_smoothed(w);
  return curvature_at(s, x, y, z);
}

/* Flux classes for the forced fill/empty rule (Sec. 2.2 cites Thuerey for it;
 * a reading, pinned by the direction of the mass it moves): an interface cell with no liquid neighbour should
 * empty (NOLIQ), one with no gas neighbour should fill (NOGAS); one with both
 * or neither is standard. */
static int flux_class(const orc_sim* s, int x, int y, int z) {
  int has_liq = 0, has_gas = 0;
  for (int i = 1; i < s->q; ++i) {
    long j;
    int t = lookup(s, x, y, z, CV[i][0], CV[i][1], CV[i][2], &j);
    if (t == ORC_LIQUID) has_liq = 1;
    if (t == ORC_GAS) has_gas = 1;
  }
  if (!has_liq && has_gas) return CLS_NOLIQ;
  if (!has_gas && has_liq) return CLS_NOGAS;
  return CLS_STD;
}

int orc_thurey_class(const orc_sim* s, int x, int y, int z) { return flux_class(s, x, y, z); }

/* Mass-flux term between interface cells with the forced fill/empty rule:
 * in = f*_ibar(nb), out = f*_i(x). Equal classes exchange in - out; a cell that
 * should fill only receives, one that should empty only sends. The table is
 * antisymmetric in (x, nb), so total mass is unchanged. */
static double thurey_term(int cx, int cn, double in, double out) {
  if (cx == cn) return in - out;
  if (cn == CLS_NOLIQ) return in;                   /* x STD or NOGAS, nb empties */
  if (cx == CLS_NOGAS && cn == CLS_STD) return in;  /* x fills */
  if (cx == CLS_NOLIQ) return -out;                 /* x empties, nb STD or NOGAS */
  return -out;                                      /* x STD, nb NOGAS fills */
}

/* ---------------------------------------------------------------------------
 * Creation.
 * ------------------------------------------------------------------------- */
static void* xcalloc(long n, long sz) { return calloc((size_t)n, (size_t)sz); }

void orc_destroy(orc_sim* s) {
  if (!s) return;
  free(s->type);
  free(s->f);
  free(s->fs);
  free(s->fn);
  free(s->m);
  free(s->phi);
  free(s->ut);
  free(s->rhoG);
  free(s->rhon);
  free(s->phis);
  free(s->share);
  free(s->mark);
  free(s->conv);
  free(s->cls);
  free(s->ntype);
  free(s->blab);
  free(s->bnew);
  free(s->btgt);
  free(s->bR);
  free(s->bamt);
  free(s->bpr);
  free(s->bpc);
  free(s->bV);
  free(s->bW);
  free(s->bnn);
  free(s->bhas);
  free(s->bqueue);
  free(s);
}

/* ---------------------------------------------------------------------------
 * Tracked bubbles (bubble_model 2). The paper follows the volume pressure of
 * each enclosed gas volume through coalescence and segmentation (Sec. 2.2,
 * volume-pressure equation and the bubble model it cites) without stating
 * the rules. Reading used here: a bubble is a connected set of gas and
 * interface cells, neighbours being the lattice directions (across periodic
 * faces; walls and obstacles separate); its volume V is the sum of 1 - phi
 * over its cells; its gas amount n = p^V V is what the volume-pressure
 * equation keeps constant (Boyle's law). After each step the bubbles are
 * found again; every old bubble hands its amount to the new bubbles holding
 * its former cells, in proportion to the gas volume of those cells
 * (coalescence adds amounts; a bubble that splits leaves each part at its
 * pressure), cells that were in no bubble add volume only, and a new bubble
 * holding none of an old bubble's volume starts at p^V(0). p^V = n / V
 * (p^V(0) where V <= 0). A bubble is labelled by its smallest cell index.
 * The hand-over n_C = sum_b n_b w_bC / W_b (w_bC: volume of b's former cells
 * now in C, W_b = sum_C w_bC) is summed so that a bubble that neither merges
 * nor splits keeps its amount exactly: of each old bubble, the new bubble
 * with the smallest label among its former cells receives the rest,
 * n_b (1 - R_b / W_b), R_b being the volume of b's former cells elsewhere,
 * and every other new bubble the shares of its cells.
 * ------------------------------------------------------------------------- */
static int is_bubble_cell(int t) { return t == ORC_GAS || t == ORC_INTERFACE; }

/* Connected components of gas and interface cells, breadth first from the
 * lowest unlabelled cell (which is then the component's smallest index). */
static void label_bubbles(const orc_sim* s, int32_t* lab, long* queue) {
  long N = s->N;
  for (long c = 0; c < N; ++c) lab[c] = -1;
  for (long c = 0; c < N; ++c) {
    if (!is_bubble_cell(s->type[c]) || lab[c] >= 0) continue;
    long head = 0, tail = 0;
    lab[c] = (int32_t)c;
    queue[tail++] = c;
    while (head < tail) {
      long a = queue[head++];
      int x, y, z;
      coords(s, a, &x, &y, &z);
      for (int i = 1; i < s->q; ++i) {
        long j;
        int t = lookup(s, x, y, z, CV[i][0], CV[i][1], CV[i][2], &j);
        if (j < 0 || !is_bubble_cell(t) || lab[j] >= 0) continue;
        lab[j] = (int32_t)c;
        queue[tail++] = j;
      }
    }
  }
}

/* Gas volume a bubble cell contributes (gas cells hold phi = 0). */
static double gas_volume(const orc_sim* s, long c) { return 1.0 - s->phi[c]; }

/* New bubbles, their amounts and pressures from the types and fill levels
 * of the end of a step; `first`: no old bubbles (creation). */
static void update_bubbles(orc_sim* s, int first) {
  long N = s->N;
  int32_t* nl = s->bnew;
  label_bubbles(s, nl, s->bqueue);
  for (long c = 0; c < N; ++c) {
    s->bV[c] = 0.0;
    s->bW[c] = 0.0;
    s->bR[c] = 0.0;
    s->bnn[c] = 0.0;
    s->bhas[c] = 0;
    s->btgt[c] = -1;
  }
  /* V of each new bubble; W of each old bubble: the gas volume of its
   * former cells that are still bubble cells; its target: the smallest new
   * label among them */
  for (long c = 0; c < N; ++c) {
    if (nl[c] < 0) continue;
    s->bV[nl[c]] += gas_volume(s, c);
    if (first || s->blab[c] < 0) continue;
    long b = s->blab[c];
    s->bW[b] += gas_volume(s, c);
    if (s->btgt[b] < 0 || nl[c] < s->btgt[b]) s->btgt[b] = nl[c];
  }
  /* amounts: through each former cell outside the target, n_b w / W_b;
   * R_b collects those cells' volume */
  for (long c = 0; c < N; ++c) {
    if (nl[c] < 0 || first || s->blab[c] < 0) continue;
    long b = s->blab[c];
    if (!(s->bW[b] > 0.0)) continue;
    s->bhas[nl[c]] = 1;
    if (nl[c] == s->btgt[b]) continue;
    s->bnn[nl[c]] += s->bamt[b] * (gas_volume(s, c) / s->bW[b]);
    s->bR[b] += gas_volume(s, c);
  }
  /* the target receives the rest of the old bubble's amount */
  for (long b = 0; b < N; ++b) {
    if (s->btgt[b] < 0 || !(s->bW[b] > 0.0)) continue;
    s->bnn[s->btgt[b]] += s->bamt[b] * (1.0 - s->bR[b] / s->bW[b]);
  }
  for (long c = 0; c < N; ++c) {
    if (nl[c] != c) continue;
    double n = s->bhas[c] ? s->bnn[c] : s->pV0 * s->bV[c];
    s->bamt[c] = n;
    s->bpr[c] = s->bV[c] > 0.0 ? n / s->bV[c] : s->pV0;
  }
  for (long c = 0; c < N; ++c) {
    s->blab[c] = nl[c];
    s->bpc[c] = nl[c] >= 0 ? s->bpr[nl[c]] : s->pV0;
  }
}

int64_t orc_bubbles(const orc_sim* s, int64_t* label, double* volume, double* pressure, int64_t cap) {
  if (s->p.bubble_model != 2) return 0;
  int64_t n = 0;
  for (long c = 0; c < s->N; ++c) {
    if (s->blab[c] != c) continue;
    if (n < cap) {
      label[n] = c;
      volume[n] = s->bV[c];
      pressure[n] = s->bpr[c];
    }
    n += 1;
  }
  return n;
}

static double bubble_volume(const orc_sim* s) {
  double V = 0.0;
  for (long c = 0; c < s->N; ++c) {
    int t = s->type[c];
    if (t == ORC_GAS)
      V += 1.0;
    else if (t == ORC_INTERFACE)
      V += 1.0 - s->phi[c];
  }
  return V;
}

int orc_create(const orc_params* p, const uint8_t* type, const double* phi, const double* rho,
               const double* ux, const double* uy, const double* uz, orc_sim** out) {
  *out = NULL;
  if (!p || p->nx < 1 || p->ny < 1 || p->nz < 1 || (p->q != 19 && p->q != 27)) return ORC_EINVAL;
  if (!(p->tau > 0.5) || (p->collision != ORC_SRT && p->collision != ORC_TRT)) return ORC_EINVAL;
  if (p->variant < ORC_NBRC || p->variant > ORC_OM3) return ORC_EINVAL;
  if (p->bubble_model < 0 || p->bubble_model > 2) return ORC_EINVAL;
  orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
  if (!s) return ORC_ENOMEM;
  s->p = *p;
  /* small domains run on one thread: the fork/join of a loop costs more
   * than the loop (the result does not depend on the count) */
  s->threads = (long)p->nx * p->ny * p->nz < 65536 ? 1 : omp_get_max_threads();
  if (s->p.tie_delta <= 0.0) s->p.tie_delta = 1e-9;
  s->q = p->q;
  s->N = (long)p->nx * p->ny * p->nz;
  long N = s->N, q = s->q;
  s->type = (uint8_t*)xcalloc(N, 1);
  s->f = (double*)xcalloc(q * N, 8);
  s->fs = (double*)xcalloc(q * N, 8);
  s->fn = (double*)xcalloc(q * N, 8);
  s->m = (double*)xcalloc(N, 8);
  s->phi = (double*)xcalloc(N, 8);
  s->ut = (double*)xcalloc(3 * N, 8);
  s->rhoG = (double*)xcalloc(N, 8);
  s->rhon = (double*)xcalloc(N, 8);
  s->phis = (double*)xcalloc(N, 8);
  s->share = (double*)xcalloc(N, 8);
  s->mark = (uint8_t*)xcalloc(N, 1);
  s->conv = (uint8_t*)xcalloc(N, 1);
  s->cls = (uint8_t*)xcalloc(N, 1);
  s->ntype = (uint8_t*)xcalloc(N, 1);
  if (!s->type || !s->f || !s->fs || !s->fn || !s->m || !s->phi || !s->ut || !s->rhoG ||
      !s->rhon || !s->phis || !s->share || !s->mark || !s->conv || !s->cls || !s->ntype) {
    orc_destroy(s);
    return ORC_ENOMEM;
  }
  memcpy(s->type, type, (size_t)N);
  for (long c = 0; c < N; ++c) {
    int t = type[c];
    if (t > ORC_FREESLIP) {
      orc_destroy(s);
      return ORC_EINVAL;
    }
    if (t == ORC_LIQUID) s->phi[c] = 1.0;
    if (t == ORC_INTERFACE) s->phi[c] = phi[c];
  }
  /* closed interface layer: no liquid cell may touch a gas cell */
  for (long c = 0; c < N; ++c) {
    if (type[c] != ORC_LIQUID) continue;
    int x, y, z;
    coords(s, c, &x, &y, &z);
    for (int i = 1; i < s->q; ++i) {
      long j;
      if (lookup(s, x, y, z, CV[i][0], CV[i][1], CV[i][2], &j) == ORC_GAS) {
        orc_destroy(s);
        return ORC_EINVAL;
      }
    }
  }
  for (long c = 0; c < N; ++c) {
    if (!is_fluid(type[c])) continue;
    double u[3] = {ux[c], uy[c], uz[c]}, feq[27];
    orc_equilibrium(s->q, rho[c], u, feq);
    for (int i = 0; i < s->q; ++i) s->f[i * N + c] = feq[i];
    if (type[c] == ORC_INTERFACE) s->m[c] = phi[c] * rho[c];
  }
  s->pV0 = s->pV = p->rho_gas / 3.0;
  s->V0 = bubble_volume(s);
  if (p->bubble_model == 2) {
    s->blab = (int32_t*)xcalloc(N, 4);
    s->bnew = (int32_t*)xcalloc(N, 4);
    s->btgt = (int32_t*)xcalloc(N, 4);
    s->bR = (double*)xcalloc(N, 8);
    s->bamt = (double*)xcalloc(N, 8);
    s->bpr = (double*)xcalloc(N, 8);
    s->bpc = (double*)xcalloc(N, 8);
    s->bV = (double*)xcalloc(N, 8);
    s->bW = (double*)xcalloc(N, 8);
    s->bnn = (double*)xcalloc(N, 8);
    s->bhas = (uint8_t*)xcalloc(N, 1);
    s->bqueue = (long*)xcalloc(N, sizeof(long));
    if (!s->blab || !s->bnew || !s->btgt || !s->bR || !s->bamt || !s->bpr || !s->bpc || !s->bV || !s->bW || !s->bnn ||
        !s->bhas || !s->bqueue) {
      orc_destroy(s);
      return ORC_ENOMEM;
    }
    update_bubbles(s, 1);
  }
  *out = s;
  return ORC_OK;
}

int orc_set_variant(orc_sim* s, int variant) {
  if (variant < ORC_NBRC || variant > ORC_OM3) return ORC_EINVAL;
  s->p.variant = variant;
  return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * One time step. Sub-steps, in this order:
 *  S1  collide every liquid and interface cell (Sec. 2.1/2.2), keep u_t;
 *  S2  normals of interface cells where a variant needs them (Sec. 2.2, 3);
 *  S3  gas density rhoG = 3 (p^V + sigma kappa) (Sec. 2.2, gas/Laplace/volume pressure);
 *  S4  pull streaming, walls, anti-bounce-back condition with the variant's set;
 *  S5  mass exchange of interface cells from post-collision populations at t;
 *  S6  density after streaming and fill level phi = m / rho;
 *  S7  conversion marks phi > 1 + eps (to liquid), phi < -eps (to gas);
 *  S8  conflicts: a to-gas mark next to a to-liquid mark is dropped;
 *  S9  new types; gas next to a to-liquid cell and liquid next to a to-gas
 *      cell become interface;
 *  S10 new interface cells from gas get feq(mean rho, mean u) of their liquid
 *      and old interface neighbours;
 *  S11 excess mass of converted cells, spread evenly over the interface
 *      neighbours after conversion (lost-mass counter if there are none);
 *  S12 fill levels of interface cells;
 *  S13 bubble volume and volume pressure (one enclosed bubble, or tracked bubbles);
 *  S14 stability checks.
 * ------------------------------------------------------------------------- */
static void collide_all(orc_sim* s, const double* f, double* fs, double* ut) {
  long N = s->N;
  int q = s->q;
#pragma omp parallel for num_threads(s->threads) schedule(static)
  for (long c = 0; c < N; ++c) {
    double fl[27], fo[27], u[3];
    if (!is_fluid(s->type[c])) {
      for (int i = 0; i < q; ++i) fs[i * N + c] = 0.0;
      continue;
    }
    for (int i = 0; i < q; ++i) fl[i] = f[i * N + c];
    orc_collide_cell(q, s->p.collision, s->p.tau, s->p.trt_lambda, s->p.smagorinsky, s->p.gravity,
                     fl, fo, u, NULL);
    for (int i = 0; i < q; ++i) fs[i * N + c] = fo[i];
    if (ut) {
      ut[3 * c + 0] = u[0];
      ut[3 * c + 1] = u[1];
      ut[3 * c + 2] = u[2];
    }
  }
}

/* Where the population arriving at cell (x,y,z) in direction i comes from.
 * Plain source: the cell x - c_i, same direction. No-slip obstacle: bounce-back
 * of the cell's own opposite population (Sec. 2.1). Free-slip obstacle
 * (Sec. 2.1: the wall-normal velocity component is reversed): the wall-normal
 * axes are those along which the one-axis step back from x is an obstacle; the
 * population comes from y = x - c_i shifted back across those axes, travelling
 * with c_j = c_i mirrored in them. No such axis, or an obstacle at y, falls back
 * to bounce-back; gas at y takes the free-surface condition (Sec. 2.2). The
 * edge/corner rules are a reading (pinned by tangential momentum conservation
 * along free-slip faces and edges).
 * Returns SRC_FLUID (with *src, *dir), SRC_GAS or SRC_BOUNCE; *via_wall tells
 * whether the direct source x - c_i is an obstacle. */
enum { SRC_FLUID = 0, SRC_GAS = 1, SRC_BOUNCE = 2 };

static int resolve_source(const orc_sim* s, int x, int y, int z, int i, long* src, int* dir,
                          int* via_wall) {
  long j;
  int st = lookup(s, x, y, z, -CV[i][0], -CV[i][1], -CV[i][2], &j);
  *via_wall = is_obstacle(st);
  *dir = i;
  *src = j;
  if (st == ORC_GAS) return SRC_GAS;
  if (is_fluid(st)) return SRC_FLUID;
  if (st == ORC_NOSLIP) return SRC_BOUNCE;
  int d[3] = {-CV[i][0], -CV[i][1], -CV[i][2]};
  int cj[3] = {CV[i][0], CV[i][1], CV[i][2]};
  int any = 0;
  for (int a = 0; a < 3; ++a) {
    if (CV[i][a] == 0) continue;
    int e[3] = {0, 0, 0};
    long k;
    e[a] = -CV[i][a];
    if (is_obstacle(lookup(s, x, y, z, e[0], e[1], e[2], &k))) {
      d[a] += CV[i][a];
      cj[a] = -CV[i][a];
      any = 1;
    }
  }
  if (!any) return SRC_BOUNCE;
  long yi;
  int ty = lookup(s, x, y, z, d[0], d[1], d[2], &yi);
  if (is_obstacle(ty)) return SRC_BOUNCE;
  if (ty == ORC_GAS) return SRC_GAS;
  *src = yi;
  *dir = dir_index(s->q, cj[0], cj[1], cj[2]);
  return SRC_FLUID;
}

static int normal_needed(int variant, uint32_t gas_mask) {
  if (variant == ORC_NBRC || variant == ORC_NBKC) return 1;
  if (variant == ORC_OM3 && __builtin_popcount(gas_mask) < 3) return 1;
  return 0;
}

static int step_once(orc_sim* s) {
  const long N = s->N;
  const int q = s->q;
  const double* g = s->p.gravity;
  const double eps = s->p.eps_phi;

  /* S1 */
  collide_all(s, s->f, s->fs, s->ut);

  /* S3 (gas density) and flux classes, from types and fill levels at t */
  if (s->p.sigma != 0.0) update_smoothed(s);
#pragma omp parallel for num_threads(s->threads) schedule(static)
  for (long c = 0; c < N; ++c) {
    if (s->type[c] != ORC_INTERFACE) continue;
    int x, y, z;
    coords(s, c, &x, &y, &z);
    double kappa = s->p.sigma != 0.0 ? curvature_at(s, x, y, z) : 0.0;
    const double pv = s->p.bubble_model == 2 ? s->bpc[c] : s->pV;
    s->rhoG[c] = 3.0 * (pv + s->p.sigma * kappa);
    s->cls[c] = (uint8_t)flux_class(s, x, y, z);
  }

  /* S2 + S4 */
  int broken = 0; /* a liquid cell next to gas: the interface layer is broken */
#pragma omp parallel for num_threads(s->threads) schedule(static)
  for (long c = 0; c < N; ++c) {
    int t = s->type[c];
    if (!is_fluid(t)) {
      for (int i = 0; i < q; ++i) s->fn[i * N + c] = 0.0;
      continue;
    }
    int x, y, z;
    coords(s, c, &x, &y, &z);
    const double* u = &s->ut[3 * c];
    uint8_t R[27];
    memset(R, 0, sizeof R);
    double rg = 0.0;
    if (t == ORC_INTERFACE) {
      uint32_t gas_mask = 0;
      for (int i = 1; i < q; ++i) {
        long j;
        if (lookup(s, x, y, z, -CV[i][0], -CV[i][1], -CV[i][2], &j) == ORC_GAS)
          gas_mask |= 1u << i;
      }
      double n[3] = {0.0, 0.0, 0.0};
      if (normal_needed(s->p.variant, gas_mask)) normal_of(s, s->phi, x, y, z, n);
      orc_reconstruct_set(q, s->p.variant, n, gas_mask, s->p.tie_delta, R);
      rg = s->rhoG[c];
    }
    for (int i = 0; i < q; ++i) {
      int ib = orc_opposite(q, i);
      long j;
      int dir, wall;
      int kind = resolve_source(s, x, y, z, i, &j, &dir, &wall);
      double v;
      if (kind == SRC_BOUNCE) {
        v = s->fs[ib * N + c];
      } else if (kind == SRC_GAS || (R[i] && !wall)) {
        /* missing population, or one the variant overwrites; populations
         * coming off a wall are never overwritten */
        if (t != ORC_INTERFACE) {
#pragma omp atomic write
          broken = 1;
        }
        v = orc_bc_value(q, i, rg, u, s->fs[ib * N + c]);
      } else {
        v = s->fs[dir * N + j];
      }
      s->fn[i * N + c] = v;
    }
  }
  if (broken) return ORC_EINVAL;

  /* S5: mass exchange, Sec. 2.2 mass-flux equation, written per arriving
   * direction k: the cell receives f*_k of the cell the population streams from
   * and gives away its own f*_kbar, which streams there. For a plain neighbour
   * nb = x - c_k this is the printed term for direction kbar; along a specular
   * reflection at a free-slip wall the partner is the reflecting cell, so that
   * the exchanged mass is exactly the exchanged populations. Operands are the
   * post-collision populations at t, types and fill levels at t; gas and
   * obstacle partners exchange nothing. */
#pragma omp parallel for num_threads(s->threads) schedule(static)
  for (long c = 0; c < N; ++c) {
    if (s->type[c] != ORC_INTERFACE) continue;
    int x, y, z;
    coords(s, c, &x, &y, &z);
    double dm = 0.0;
    for (int k = 1; k < q; ++k) {
      long j;
      int dir, wall;
      if (resolve_source(s, x, y, z, k, &j, &dir, &wall) != SRC_FLUID) continue;
      double in = s->fs[dir * N + j];
      double out = s->fs[orc_opposite(q, k) * N + c];
      if (s->type[j] == ORC_LIQUID) {
        dm += in - out;
      } else {
        double T = s->p.thurey_flux ? thurey_term(s->cls[c], s->cls[j], in, out) : in - out;
        dm += 0.5 * (s->phi[c] + s->phi[j]) * T;
      }
    }
    s->m[c] += dm;
  }

  /* S6 + S7 */
#pragma omp parallel for num_threads(s->threads) schedule(static)
  for (long c = 0; c < N; ++c) {
    s->mark[c] = MARK_NONE;
    s->conv[c] = CONV_NONE;
    if (!is_fluid(s->type[c])) continue;
    double r = 0.0;
    for (int i = 0; i < q; ++i) r += s->fn[i * N + c];
    s->rhon[c] = r;
    if (s->type[c] == ORC_INTERFACE) {
      double ph = s->m[c] / r;
      s->phi[c] = ph;
      if (ph > 1.0 + eps)
        s->mark[c] = MARK_L;
      else if (ph < -eps)
        s->mark[c] = MARK_G;
    }
  }

  /* S8: separation of liquid and gas takes priority, so a cell that would
   * empty next to one that fills stays interface. */
  for (long c = 0; c < N; ++c) {
    if (s->mark[c] != MARK_G) continue;
    int x, y, z;
    coords(s, c, &x, &y, &z);
    for (int i = 1; i < q; ++i) {
      long j;
      int t = lookup(s, x, y, z, CV[i][0], CV[i][1], CV[i][2], &j);
      if (t == ORC_INTERFACE && s->mark[j] == MARK_L) {
        s->mark[c] = MARK_NONE;
        break;
      }
    }
  }

  /* S9: new types (liquid and gas never convert into one another directly) */
#pragma omp parallel for num_threads(s->threads) schedule(static)
  for (long c = 0; c < N; ++c) {
    int t = s->type[c];
    s->ntype[c] = (uint8_t)t;
    if (t == ORC_INTERFACE) {
      if (s->mark[c] == MARK_L) {
        s->ntype[c] = ORC_LIQUID;
        s->conv[c] = CONV_TO_LIQ;
      } else if (s->mark[c] == MARK_G) {
        s->ntype[c] = ORC_GAS;
        s->conv[c] = CONV_TO_GAS;
      }
    } else if (t == ORC_GAS || t == ORC_LIQUID) {
      int want = (t == ORC_GAS) ? MARK_L : MARK_G;
      int x, y, z;
      coords(s, c, &x, &y, &z);
      for (int i = 1; i < q; ++i) {
        long j;
        int tn = lookup(s, x, y, z, CV[i][0], CV[i][1], CV[i][2], &j);
        if (tn == ORC_INTERFACE && s->mark[j] == want) {
          s->ntype[c] = ORC_INTERFACE;
          s->conv[c] = (t == ORC_GAS) ? CONV_NEW_FROM_GAS : CONV_NEW_FROM_LIQ;
          break;
        }
      }
    }
  }

  /* S10: populations of new interface cells from gas: equilibrium with the
   * arithmetic mean density and velocity of the liquid and non-new interface
   * neighbours (velocity with the half-force shift, as in Sec. 2.1). Only
   * cells that are not new from gas are read, only such cells are written. */
#pragma omp parallel for num_threads(s->threads) schedule(static)
  for (long c = 0; c < N; ++c) {
    if (s->conv[c] != CONV_NEW_FROM_GAS) continue;
    int x, y, z;
    coords(s, c, &x, &y, &z);
    double rs = 0.0, us[3] = {0.0, 0.0, 0.0};
    int cnt = 0;
    for (int i = 1; i < q; ++i) {
      long j;
      lookup(s, x, y, z, CV[i][0], CV[i][1], CV[i][2], &j);
      if (j < 0) continue;
      int nt = s->ntype[j];
      if (!is_fluid(nt) || s->conv[j] == CONV_NEW_FROM_GAS) continue;
      double r, u[3];
      moments(q, &s->fn[j], N, g, &r, u);
      rs += r;
      us[0] += u[0];
      us[1] += u[1];
      us[2] += u[2];
      cnt += 1;
    }
    double rbar = rs / cnt;
    double ubar[3] = {us[0] / cnt, us[1] / cnt, us[2] / cnt};
    double feq[27];
    orc_equilibrium(q, rbar, ubar, feq);
    for (int i = 0; i < q; ++i) s->fn[i * N + c] = feq[i];
    s->rhon[c] = rbar;
    s->m[c] = 0.0;
  }
#pragma omp parallel for num_threads(s->threads) schedule(static)
  for (long c = 0; c < N; ++c)
    if (s->conv[c] == CONV_NEW_FROM_LIQ) s->m[c] = s->rhon[c];

  /* S11: excess mass, Sec. 2.2 excess-mass equation (m_ex = m - rho when
   * filled, m when emptied), equal shares to the interface neighbours after
   * conversion; each receiver adds its shares in direction order. */
  for (long c = 0; c < N; ++c) {
    if (s->conv[c] != CONV_TO_LIQ && s->conv[c] != CONV_TO_GAS) continue;
    int x, y, z;
    coords(s, c, &x, &y, &z);
    int nif = 0;
    for (int i = 1; i < q; ++i) {
      long j;
      lookup(s, x, y, z, CV[i][0], CV[i][1], CV[i][2], &j);
      if (j >= 0 && s->ntype[j] == ORC_INTERFACE) nif += 1;
    }
    double mex = s->conv[c] == CONV_TO_LIQ ? s->m[c] - s->rhon[c] : s->m[c];
    if (nif == 0) {
      s->m_lost += mex;
      s->share[c] = 0.0;
    } else {
      s->share[c] = mex / nif;
    }
  }
#pragma omp parallel for num_threads(s->threads) schedule(static)
  for (long c = 0; c < N; ++c) {
    if (s->ntype[c] != ORC_INTERFACE) continue;
    int x, y, z;
    coords(s, c, &x, &y, &z);
    for (int i = 1; i < q; ++i) {
      long j;
      lookup(s, x, y, z, CV[i][0], CV[i][1], CV[i][2], &j);
      if (j < 0) continue;
      if (s->conv[j] == CONV_TO_LIQ || s->conv[j] == CONV_TO_GAS) s->m[c] += s->share[j];
    }
  }

  /* S12: fill levels and the new state */
#pragma omp parallel for num_threads(s->threads) schedule(static)
  for (long c = 0; c < N; ++c) {
    int nt = s->ntype[c];
    s->type[c] = (uint8_t)nt;
    if (nt == ORC_INTERFACE) {
      s->phi[c] = s->m[c] / s->rhon[c];
    } else if (nt == ORC_LIQUID) {
      s->phi[c] = 1.0;
      s->m[c] = 0.0;
    } else if (nt == ORC_GAS) {
      s->phi[c] = 0.0;
      s->m[c] = 0.0;
    }
    if (is_fluid(nt)) {
      for (int i = 0; i < q; ++i) s->f[i * N + c] = s->fn[i * N + c];
    } else {
      for (int i = 0; i < q; ++i) s->f[i * N + c] = 0.0;
    }
  }

  /* S13: Sec. 2.2 volume pressure p^V = p^V(0) V(0)/V(t): one enclosed
   * bubble, or every bubble tracked through coalescence and segmentation */
  if (s->p.bubble_model == 1) s->pV = s->pV0 * s->V0 / bubble_volume(s);
  if (s->p.bubble_model == 2) update_bubbles(s, 0);

  /* S14: instability (the paper observed blow-ups once the flow exceeded the
   * lattice speed of sound) */
  int unstable = 0;
#pragma omp parallel for num_threads(s->threads) schedule(static)
  for (long c = 0; c < N; ++c) {
    if (!is_fluid(s->type[c])) continue;
    double r, u[3];
    moments(q, &s->f[c], N, g, &r, u);
    double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    if (!(r > 0.0) || !isfinite(r) || !isfinite(usq) || !(usq < 1.0 / 3.0) ||
        (s->type[c] == ORC_INTERFACE && !isfinite(s->m[c]))) {
#pragma omp atomic write
      unstable = 1;
    }
  }
  if (unstable) return ORC_EUNSTABLE;
  s->step += 1;
  return ORC_OK;
}

int orc_step(orc_sim* s, int64_t n) {
  if (s->status != ORC_OK) return s->status;
  for (int64_t k = 0; k < n; ++k) {
    int st = step_once(s);
    if (st != ORC_OK) {
      s->status = st;
      return st;
    }
  }
  return ORC_OK;
}

void orc_fields(const orc_sim* s, uint8_t* type, double* phi, double* rho, double* ux, double* uy,
                double* uz, double* mass, double* pdf) {
  long N = s->N;
  int q = s->q;
  for (long c = 0; c < N; ++c) {
    int t = s->type[c];
    if (type) type[c] = (uint8_t)t;
    if (phi) phi[c] = s->phi[c];
    double r = 0.0, u[3] = {0.0, 0.0, 0.0};
    if (is_fluid(t)) moments(q, &s->f[c], N, s->p.gravity, &r, u);
    if (rho) rho[c] = r;
    if (ux) ux[c] = u[0];
    if (uy) uy[c] = u[1];
    if (uz) uz[c] = u[2];
    if (mass) mass[c] = t == ORC_INTERFACE ? s->m[c] : (t == ORC_LIQUID ? r : 0.0);
  }
  if (pdf) memcpy(pdf, s->f, sizeof(double) * (size_t)q * (size_t)N);
}

void orc_post_collision(const orc_sim* s, double* pdf_star) {
  collide_all((orc_sim*)s, s->f, pdf_star, NULL);
}

int orc_set_threads(orc_sim* s, int threads) {
  if (threads < 1) return ORC_EINVAL;
  s->threads = threads;
  return ORC_OK;
}

void orc_export_state(const orc_sim* s, uint8_t* type, double* pdf, double* mass, double* phi,
                      double scalars[4]) {
  long N = s->N;
  if (type) memcpy(type, s->type, (size_t)N);
  if (pdf) memcpy(pdf, s->f, sizeof(double) * (size_t)s->q * (size_t)N);
  if (mass) memcpy(mass, s->m, sizeof(double) * (size_t)N);
  if (phi) memcpy(phi, s->phi, sizeof(double) * (size_t)N);
  if (scalars) {
    scalars[0] = s->m_lost;
    scalars[1] = s->pV;
    scalars[2] = s->pV0;
    scalars[3] = s->V0;
  }
}

int orc_import_state(orc_sim* s, const uint8_t* type, const double* pdf, const double* mass,
                     const double* phi, const double scalars[4], int64_t step) {
  long N = s->N;
  for (long c = 0; c < N; ++c)
    if (type[c] > ORC_FREESLIP) return ORC_EINVAL;
  memcpy(s->type, type, (size_t)N);
  memcpy(s->f, pdf, sizeof(double) * (size_t)s->q * (size_t)N);
  memcpy(s->m, mass, sizeof(double) * (size_t)N);
  memcpy(s->phi, phi, sizeof(double) * (size_t)N);
  s->m_lost = scalars[0];
  s->pV = scalars[1];
  s->pV0 = scalars[2];
  s->V0 = scalars[3];
  s->step = step;
  s->status = ORC_OK;
  /* tracked bubbles restart from the imported types: every bubble at p^V(0) */
  if (s->p.bubble_model == 2) update_bubbles(s, 1);
  return ORC_OK;
}

void orc_mass(const orc_sim* s, orc_report* r) {
  memset(r, 0, sizeof *r);
  long N = s->N;
  for (long c = 0; c < N; ++c) {
    int t = s->type[c];
    if (t == ORC_LIQUID) {
      double rho = 0.0;
      for (int i = 0; i < s->q; ++i) rho += s->f[i * N + c];
      r->liquid_mass += rho;
      r->n_liquid += 1;
    } else if (t == ORC_INTERFACE) {
      r->interface_mass += s->m[c];
      r->n_interface += 1;
    } else if (t == ORC_GAS) {
      r->n_gas += 1;
    }
  }
  r->lost_mass = s->m_lost;
  r->total_mass = r->liquid_mass + r->interface_mass + r->lost_mass;
  r->bubble_volume = bubble_volume(s);
  r->p_volume = s->pV;
  r->step = s->step;
}
