/* Host-side paths of the C ABI, driven from plain C without a GPU: parameter
 * validation, footprints and layouts, argument checks that return before any
 * device access, and the handles' null cases.  Built against a host-only copy
 * of the library with AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_host_sanitizers.py; exits 0 and prints "ok" when every check
 * holds, 1 at the first that does not. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "picmcc.h"

static int failures = 0;
#define CHECK(cond)                                                   \
  do {                                                                \
    if (!(cond)) {                                                    \
      fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
      ++failures;                                                     \
    }                                                                 \
  } while (0)

/* the small discharge: 25 mm, 64 cells, 100 V at 13.56 MHz, Ar 1 Pa, 5k + 5k */
static pm_case_params small_case(void) {
  pm_case_params p;
  memset(&p, 0, sizeof(p));
  p.gap_m = 0.025;
  p.n_cells = 64;
  p.steps_per_cycle = 400;
  p.freq_hz = 13.56e6;
  p.v0_volt = 100.0;
  p.phase_rad = -M_PI / 2;
  p.p_pa = 1.0;
  p.t_gas_k = 300.0;
  p.n0_m3 = 1e15;
  p.np_e = p.np_i = 5000;
  p.te_ev = 2.0;
  p.ti_ev = 0.026;
  p.capacity_e = p.capacity_i = 20000;
  p.ecap_e_ev = p.ecap_i_ev = 300.0;
  p.xs.sigma_el = 1e-19;
  p.xs.eth_exc = 11.5;
  p.xs.sigma0_exc = 2.5e-20;
  p.xs.eth_ion = 15.8;
  p.xs.sigma0_ion = 2.5e-20;
  p.xs.sigma_cx = 5e-19;
  p.seed = 1234;
  p.case_id = 1;
  p.fp64 = 1;
  p.sort_interval = 25;
  return p;
}

static pm_tp_params flight(void) {
  pm_tp_params t;
  memset(&t, 0, sizeof(t));
  t.p_pa = 0.5;
  t.t_gas_k = 300.0;
  t.d_ref = 3.6e-10;
  t.omega = 0.8;
  t.t_ref = 273.0;
  t.m_test_amu = 26.9815385;
  t.m_gas_amu = 39.948;
  t.gap_m = 0.04;
  t.lateral_m = 0.1;
  t.mode = PM_TP_NORMAL;
  t.e_max = 1000000;
  t.n_ebins = 200;
  t.ebin_ev = 1.0;
  t.n_tbins = 200;
  t.tbin_s = 5e-6;
  t.n_xbins = 100;
  return t;
}

int main(void) {
  for (int s = -8; s <= 1; ++s) CHECK(pm_status_string((pm_status)s) != NULL);

  /* footprints of valid cases grow with the grid, the slots and the sums */
  pm_case_params p = small_case();
  const size_t base = pm_case_footprint(&p);
  CHECK(base > 0);
  pm_case_params q = p;
  q.fp64 = 0;
  CHECK(pm_case_footprint(&q) > 0 && pm_case_footprint(&q) < base);
  q = p;
  q.n_cells = 1024;
  CHECK(pm_case_footprint(&q) > base);
  q = p;
  q.n_cells = 1;
  CHECK(pm_case_footprint(&q) > 0);
  q = p;
  q.n_phase = 128;
  q.steps_per_cycle = 400;
  q.flux_profiles = 1;
  q.v2_volt = 100.0;
  q.cb_f_m2 = 1e-8;
  CHECK(pm_case_footprint(&q) > base);
  q = p;
  q.np_e = q.np_i = 1000000;
  q.capacity_e = q.capacity_i = 4000000;
  CHECK(pm_case_footprint(&q) > (size_t)2 * 2 * 4000000 * 28);
  q = p;
  q.capacity_e = q.capacity_i = INT32_MAX;
  CHECK(pm_case_footprint(&q) > (size_t)INT32_MAX);

  /* invalid parameters: footprint 0, init refused */
  pm_case_params bad[16];
  int nb = 0;
  bad[nb] = p; bad[nb++].n_cells = 0;
  bad[nb] = p; bad[nb++].n_cells = 1025;
  bad[nb] = p; bad[nb++].steps_per_cycle = 0;
  bad[nb] = p; bad[nb++].np_e = 0;
  bad[nb] = p; bad[nb++].capacity_e = 10;
  bad[nb] = p; bad[nb++].capacity_i = (int64_t)INT32_MAX + 1;
  bad[nb] = p; bad[nb++].fp64 = 3;
  bad[nb] = p; bad[nb++].gap_m = -1.0;
  bad[nb] = p; bad[nb++].v0_volt = NAN;
  bad[nb] = p; bad[nb++].p_pa = -1.0;
  bad[nb] = p; bad[nb++].sort_interval = -2;
  bad[nb] = p; bad[nb++].n_phase = 129;
  bad[nb] = p; bad[nb++].flux_profiles = 2;
  bad[nb] = p; bad[nb++].cb_f_m2 = -1.0;
  bad[nb] = p; bad[nb++].ecap_i_ev = 2e6;
  bad[nb] = p; bad[nb++].t_gas_k = 0.0;
  pm_case* h = NULL;
  for (int i = 0; i < nb; ++i) {
    CHECK(pm_case_footprint(&bad[i]) == 0);
    CHECK(pm_init_case(&bad[i], (void*)(uintptr_t)(1u << 20), base, NULL, &h) == PM_EINVAL);
    CHECK(h == NULL);
  }
  CHECK(pm_case_footprint(NULL) == 0);
  /* arguments checked before any device access */
  CHECK(pm_init_case(NULL, (void*)(uintptr_t)(1u << 20), base, NULL, &h) == PM_EINVAL);
  CHECK(pm_init_case(&p, NULL, base, NULL, &h) == PM_EINVAL);
  CHECK(pm_init_case(&p, (void*)(uintptr_t)(1u << 20), base - 1, NULL, &h) == PM_ENOSPACE);
  CHECK(pm_init_case(&p, (void*)(uintptr_t)((1u << 20) + 8), base, NULL, &h) == PM_EINVAL);
  CHECK(h == NULL);

  /* calls on no case */
  unsigned char buf[64];
  pm_diagnostics d;
  memset(&d, 0, sizeof(d));
  pm_launch_shape sh = {8, 0, 0, 1, 25, 1};
  CHECK(pm_step(NULL, 1, NULL) == PM_EINVAL);
  CHECK(pm_step_rf_cycles(NULL, 1, NULL) == PM_EINVAL);
  CHECK(pm_sample_diagnostics(NULL, &d, 0, NULL) == PM_EINVAL);
  CHECK(pm_checkpoint_bytes(NULL) == 0);
  CHECK(pm_save_checkpoint(NULL, buf, sizeof(buf), NULL) == PM_EINVAL);
  CHECK(pm_load_checkpoint(NULL, buf, sizeof(buf), NULL) == PM_EINVAL);
  CHECK(pm_philox_words(0, 0, 0, 0, 0, 0, -1, NULL, NULL) == PM_EINVAL);
  CHECK(pm_philox_words(0, 0, 0, 0, 0, 0, 5, NULL, NULL) == PM_EINVAL);
  CHECK(pm_philox_words(0, 0, 0, 0, 0, 0, 0, NULL, NULL) == PM_OK);
  CHECK(pm_set_launch_shape(NULL, &sh, NULL) == PM_EINVAL);
  CHECK(pm_get_launch_shape(NULL, &sh) == PM_EINVAL);
  pm_destroy_case(NULL);

  /* batches */
  pm_case* none[1] = {NULL};
  pm_batch* bh = NULL;
  CHECK(pm_batch_footprint(NULL, 0) == 0);
  CHECK(pm_batch_footprint(none, 1) == 0);
  CHECK(pm_batch_create(none, 1, (void*)(uintptr_t)(1u << 20), 1u << 20, NULL, &bh) == PM_EINVAL);
  CHECK(bh == NULL);
  CHECK(pm_batch_create_slots(0, 0, 400, 64, (void*)(uintptr_t)(1u << 20), 1u << 20, NULL, &bh) == PM_EINVAL);
  CHECK(pm_batch_create_slots(4, 2, 400, 64, (void*)(uintptr_t)(1u << 20), 1u << 20, NULL, &bh) == PM_EINVAL);
  CHECK(pm_batch_create_slots(4, 0, 400, 1025, (void*)(uintptr_t)(1u << 20), 1u << 20, NULL, &bh) == PM_EINVAL);
  CHECK(bh == NULL);
  CHECK(pm_batch_slots_footprint(4, 0) > 0);
  CHECK(pm_batch_step(NULL, 1, NULL) == PM_EINVAL);
  CHECK(pm_batch_step_rf_cycles(NULL, 1, NULL) == PM_EINVAL);
  CHECK(pm_batch_set_launch_shape(NULL, &sh, NULL) == PM_EINVAL);
  pm_batch_destroy(NULL);

  /* test-atom flights */
  pm_tp_params t = flight();
  const size_t tpb = pm_tp_footprint(&t);
  CHECK(tpb > 0);
  pm_tp_source src;
  memset(&src, 0, sizeof(src));
  src.n_atoms = 1000;
  src.u_s_ev = 3.4;
  src.e_cut_ev = 200.0;
  src.seed = 1234;
  src.job_id = 3;
  pm_tp_result res;
  memset(&res, 0, sizeof(res));
  pm_tp_params tb[6];
  int nt = 0;
  tb[nt] = t; tb[nt++].omega = 0.3;
  tb[nt] = t; tb[nt++].mode = 7;
  tb[nt] = t; tb[nt++].e_max = 0;
  tb[nt] = t; tb[nt++].gap_m = 0.0;
  tb[nt] = t; tb[nt++].n_xbins = 5000;
  tb[nt] = t; tb[nt++].scatter = 9;
  for (int i = 0; i < nt; ++i) {
    CHECK(pm_run_test_particles(&tb[i], &src, (void*)(uintptr_t)(1u << 20), tpb, NULL, &res) == PM_EINVAL);
    CHECK(pm_run_test_particles_static(&tb[i], &src, NULL, &res) == PM_EINVAL);
  }
  CHECK(pm_run_test_particles(&t, &src, (void*)(uintptr_t)(1u << 20), 16, NULL, &res) == PM_ENOSPACE);
  CHECK(pm_run_test_particles(NULL, &src, (void*)(uintptr_t)(1u << 20), tpb, NULL, &res) == PM_EINVAL);
  CHECK(pm_run_test_particles(&t, NULL, (void*)(uintptr_t)(1u << 20), tpb, NULL, &res) == PM_EINVAL);
  pm_tp_params big = t;
  big.n_ebins = 200000;
  CHECK(pm_tp_footprint(&big) > PM_TP_STATIC_BYTES);
  CHECK(pm_run_test_particles_static(&big, &src, NULL, &res) == PM_ENOSPACE);

  if (failures) return 1;
  printf("ok\n");
  return 0;
}
