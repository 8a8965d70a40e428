/* Flow-boiling channel through the C ABI alone (no Python): the 200x50
 * channel of the library defaults with a 20-cell heater at 1.1 T_sat,
 * 2000 steps, then the FP64 diagnostics and the temperature on the heater.
 *
 *   gcc -O2 -std=c11 channel.c -I../../include -L.. -llbmflow -Wl,-rpath,'$ORIGIN/..' -o channel
 */
#include <stdio.h>
#include <stdlib.h>

#include "lbmflow.h"

#define CHECK(call)                                                              \
  do {                                                                           \
    int rc_ = (call);                                                            \
    if (rc_ != LBM_OK) {                                                         \
      fprintf(stderr, "%s failed (%d): %s\n", #call, rc_, lbm_last_error());      \
      return 1;                                                                  \
    }                                                                            \
  } while (0)

int main(void) {
  lbm_params p;
  CHECK(lbm_params_default(&p));  /* 200x50 channel, Peng-Robinson constants of Sec. 2A */
  double rho_l, rho_v, p_sat;
  CHECK(lbm_maxwell(&p, p.T_iso, &rho_l, &rho_v, &p_sat));  /* saturation state at T_sat */
  p.storage = LBM_STORE_F32_DEV;
  p.rho_ref = rho_l;
  p.T_ref = p.T_iso;

  lbm_domain* d = NULL;
  CHECK(lbm_create(&p, NULL, NULL, 0, &d));
  double* Tw = malloc(sizeof(double) * p.nx);
  double* rw = malloc(sizeof(double) * p.nx);
  int32_t* heater = calloc(p.nx, sizeof(int32_t));
  for (int x = 0; x < p.nx; ++x) {
    heater[x] = x >= p.nx / 2 - 10 && x < p.nx / 2 + 10;
    Tw[x] = heater[x] ? 1.1 * p.T_iso : p.T_in;
    rw[x] = 3.8; /* false wall density: ~60 degree contact angle */
  }
  CHECK(lbm_set_wall_maps(d, LBM_SIDE_S, Tw, rw, heater));
  for (int x = 0; x < p.nx; ++x) Tw[x] = p.T_in;
  CHECK(lbm_set_wall_maps(d, LBM_SIDE_N, Tw, rw, NULL));
  CHECK(lbm_init_fields(d, NULL, NULL, rho_l, p.T_iso, 1e-3, 1));
  CHECK(lbm_step(d, 2000));
  CHECK(lbm_sync(d));

  lbm_diag g;
  CHECK(lbm_read_diag(d, &g));
  printf("step %lld: mass %.6f energy %.6f heater flux %.6e vapour cells %.0f\n", (long long)g.step,
         g.mass, g.energy, g.heater_q, g.vapor_cells);
  printf("heater Nusselt number %.4f, centreline pressure drop %.6e\n", g.nu_heater, g.dp);
  double* f = malloc(sizeof(double) * 4 * p.nx * p.ny);
  CHECK(lbm_read_fields(d, f, f + p.nx * p.ny, f + 2 * p.nx * p.ny, f + 3 * p.nx * p.ny));
  const double* T = f + 3 * p.nx * p.ny;
  printf("T(x = nx/2, y = 0) = %.6f (T_sat %.6f)\n", T[p.nx / 2], p.T_iso);
  CHECK(lbm_destroy(d));
  free(f);
  free(heater);
  free(rw);
  free(Tw);
  return 0;
}
