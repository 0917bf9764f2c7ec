/*
 * sanitize_driver.c -- TEST INFRASTRUCTURE: a small program that runs every
 * exported routine of the FP64 oracle (rt_oracle.c, compiled into it) on a
 * tiny synthetic case, so that the oracle can be built and run under the
 * address and undefined-behaviour sanitizers (tests/test_oracle_sanitized.py).
 * It checks nothing numerical; the sanitizers report any out-of-bounds
 * access, leak or undefined operation, and the exit status is 0 otherwise.
 */
#include "rt_oracle.c"

#include <stdio.h>

int main(void) {
  enum { NX = 3, NY = 2, NZ = 4, NC = NX * NY * NZ, NL = 9, NNU = 700, NR = 40 };
  double T[NC], x[NC], p[NC];
  for (int c = 0; c < NC; ++c) {
    T[c] = 350.0 + 60.0 * c;
    x[c] = 0.02 + 0.01 * (c % 7);
    p[c] = 0.8 + 0.05 * (c % 5);
  }
  double nu[NL], S[NL], g[NL], n[NL], E[NL];
  for (int i = 0; i < NL; ++i) {
    nu[i] = 999.0 + 0.83 * i;            /* first ones centred below the grid */
    S[i] = (i == 4) ? 0.0 : 1e-21 * (1 + i);
    g[i] = 0.05 + 0.005 * i;
    n[i] = 0.5;
    E[i] = 150.0 * i;
  }
  int32_t cells[NC];
  for (int c = 0; c < NC; ++c) cells[c] = c;
  const double nu0 = 1000.0, dnu = 0.01, cutoff = 1.0, T_ref = 296.0;
  double* out = (double*)malloc(sizeof(double) * NC * NNU);
  double* B = (double*)malloc(sizeof(double) * NC * NNU);
  int rc = 0;
  rc |= orc_kappa(NC, cells, T, x, p, NL, nu, S, g, n, E, T_ref, cutoff, nu0, dnu, NNU, out) != 0;
  rc |= orc_kappa(NC, cells, T, x, p, NL, nu, S, g, n, NULL, T_ref, cutoff, nu0, dnu, NNU, out) != 0;
  rc |= orc_kappa_table16(NC, cells, T, x, p, NL, nu, S, g, E, T_ref, nu0, dnu, NNU, out) != 0;
  rc |= orc_kappa_adaptive(NC, cells, NC, T, x, p, NL, nu, S, g, n, E, T_ref, cutoff, nu0, dnu,
                           NNU, 1e-3, 8, out) != 0;
  rc |= orc_adaptive_evals(NC, T, p, NL, nu, S, g, n, E, T_ref, cutoff, nu0, dnu, NNU, 1e-3, 8) < 0;
  (void)orc_mean_strength(T[0], NL, nu, S, E, T_ref, cutoff, nu0, dnu, NNU);
  rc |= orc_planck_rows(NC, cells, T, nu0, dnu, NNU, B) != 0;
  int64_t O[NR * 3], D[NR * 3];
  for (int r = 0; r < NR; ++r) {
    int32_t face = -1;
    rc |= orc_ray(0, (uint64_t)r, NX, NY, NZ, O + 3 * r, D + 3 * r, &face) != 0;
  }
  int32_t sc[NX + NY + NZ + 3];
  double sl[NX + NY + NZ + 3];
  for (int r = 0; r < NR; ++r)
    rc |= orc_segments(NX, NY, NZ, 5.0, O + 3 * r, D + 3 * r, sc, sl, NX + NY + NZ + 3) < 0;
  orc_kappa(NC, cells, T, x, p, NL, nu, S, g, n, E, T_ref, cutoff, nu0, dnu, NNU, out);
  double absorbed[NC] = {0}, emitted[NC] = {0}, balance[4] = {0};
  double* exit_I = (double*)malloc(sizeof(double) * NR * NNU);
  rc |= orc_march(NX, NY, NZ, 5.0, NR, O, D, 1e-3, 1200.0, nu0, dnu, NNU, out, B, NULL, absorbed,
                  emitted, balance, exit_I) != 0;
  uint64_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, w[4];
  orc_philox4x64_10(ctr, key, w);
  free(out);
  free(B);
  free(exit_I);
  printf("oracle routines ran: %s\n", rc ? "with errors" : "ok");
  return rc;
}
