/* Runs the FP64 oracle on setups written by test_oracle_readings.py, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer. Each file holds
 * 15 int32 (nx, ny, nz, q, collision, boundary[6], variant, thurey_flux,
 * bubble_model, steps), 10 doubles (tau, trt_lambda, gravity[3], rho_gas,
 * sigma, eps_phi, tie_delta, smagorinsky), N type bytes and the N-arrays
 * phi, rho, ux, uy, uz. Prints "ok" per case that steps without error. */
#include <stdio.h>
#include <stdlib.h>

#include "fslbm_oracle.h"

static int run(const char* path) {
  FILE* fh = fopen(path, "rb");
  if (!fh) return 1;
  int32_t in[15];
  double db[10];
  if (fread(in, 4, 15, fh) != 15 || fread(db, 8, 10, fh) != 10) return 2;
  orc_params p;
  p.nx = in[0];
  p.ny = in[1];
  p.nz = in[2];
  p.q = in[3];
  p.collision = in[4];
  for (int f = 0; f < 6; ++f) p.boundary[f] = in[5 + f];
  p.variant = in[11];
  p.thurey_flux = in[12];
  p.bubble_model = in[13];
  const int steps = in[14];
  p.tau = db[0];
  p.trt_lambda = db[1];
  for (int a = 0; a < 3; ++a) p.gravity[a] = db[2 + a];
  p.rho_gas = db[5];
  p.sigma = db[6];
  p.eps_phi = db[7];
  p.tie_delta = db[8];
  p.smagorinsky = db[9];
  const long N = (long)p.nx * p.ny * p.nz;
  uint8_t* type = malloc((size_t)N);
  double* a[5];
  for (int k = 0; k < 5; ++k) a[k] = malloc(sizeof(double) * (size_t)N);
  int bad = fread(type, 1, (size_t)N, fh) != (size_t)N;
  for (int k = 0; k < 5; ++k) bad |= fread(a[k], 8, (size_t)N, fh) != (size_t)N;
  fclose(fh);
  int st = bad ? 3 : 0;
  orc_sim* s = NULL;
  if (!st) st = orc_create(&p, type, a[0], a[1], a[2], a[3], a[4], &s);
  if (!st) st = orc_step(s, steps);
  if (!st) {
    orc_report r;
    orc_mass(s, &r);
    double* pdf = malloc(sizeof(double) * (size_t)p.q * (size_t)N);
    double* m = malloc(sizeof(double) * (size_t)N);
    double* phi = malloc(sizeof(double) * (size_t)N);
    double sc[4];
    orc_export_state(s, type, pdf, m, phi, sc);
    st = orc_import_state(s, type, pdf, m, phi, sc, r.step);
    if (!st) st = orc_step(s, 2);
    printf("%s ok: M = %.17g, %lld interface cells\n", path, r.total_mass, (long long)r.n_interface);
    free(pdf);
    free(m);
    free(phi);
  }
  orc_destroy(s);
  free(type);
  for (int k = 0; k < 5; ++k) free(a[k]);
  if (st) printf("%s failed: %d\n", path, st);
  return st != 0;
}

int main(int argc, char** argv) {
  int bad = 0;
  for (int i = 1; i < argc; ++i) bad |= run(argv[i]);
  return bad;
}
