/* check_main.c -- command-line runner of the oracle (test infrastructure): reads an orc_params
 * struct and the initial phi (FP64, site order x fastest) from two binary files, advances the
 * given number of steps and prints the observables.  Built with the address and undefined-
 * behaviour sanitizers by the CPU test-suite, so that any out-of-bounds access, use after free,
 * leak or undefined operation in the oracle aborts the run.
 * Usage: check_main params.bin phi0.bin steps */
#include <stdio.h>
#include <stdlib.h>

#include "lam_oracle.h"

static void* slurp(const char* path, size_t* n) {
  FILE* f = fopen(path, "rb");
  if (!f) return NULL;
  fseek(f, 0, SEEK_END);
  long len = ftell(f);
  fseek(f, 0, SEEK_SET);
  void* buf = len > 0 ? malloc((size_t)len) : NULL;
  if (buf && fread(buf, 1, (size_t)len, f) != (size_t)len) {
    free(buf);
    buf = NULL;
  }
  fclose(f);
  *n = buf ? (size_t)len : 0;
  return buf;
}

int main(int argc, char** argv) {
  if (argc != 4) {
    fprintf(stderr, "usage: %s params.bin phi0.bin steps\n", argv[0]);
    return 2;
  }
  size_t np = 0, nphi = 0;
  orc_params* p = (orc_params*)slurp(argv[1], &np);
  double* phi0 = (double*)slurp(argv[2], &nphi);
  if (!p || np != sizeof(orc_params) || !phi0) {
    fprintf(stderr, "bad input files\n");
    return 2;
  }
  long N = (long)p->nx * p->ny * (p->dim == 3 ? p->nz : 1);
  if ((long)(nphi / sizeof(double)) != N) {
    fprintf(stderr, "phi0 holds %zu values, the lattice %ld sites\n", nphi / sizeof(double), N);
    return 2;
  }
  orc_sim* s = NULL;
  if (orc_create(p, &s) != 0) return 3;
  if (orc_init_fields(s, phi0, NULL, NULL) != 0) return 3;
  if (orc_step(s, atol(argv[3])) != 0) return 3;
  orc_obs o;
  if (orc_observables(s, &o) != 0) return 3;
  /* a checkpoint round trip exercises the state functions too */
  size_t nb = orc_state_bytes(s);
  void* buf = malloc(nb);
  if (!buf || orc_get_state(s, buf, nb) != 0 || orc_set_state(s, buf, nb) != 0) return 3;
  free(buf);
  printf("%.17g %.17g %.17g %.17g %lld %d\n", o.mass_dev, o.phi_sum, o.max_u, o.free_energy,
         (long long)o.step, o.nonfinite);
  orc_destroy(s);
  free(p);
  free(phi0);
  return 0;
}
