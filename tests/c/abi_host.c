/* Host-only use of the C ABI from plain C99: spaces, a spin-blocked tensor pair, a plan of the
 * particle-particle ladder R(a,b,i,j) = 1/2 V(a,b,c,d) T(c,d,i,j), its statistics, and error codes.
 * No GPU call is made (plan creation is host-only).  Prints one line per check; exit status 0 on
 * success. */
#include <stdio.h>
#include <string.h>

#include "tamm_mi.h"

static int fails = 0;
#define CHECK(cond)                                               \
  do {                                                            \
    if (!(cond)) {                                                \
      printf("FAIL %s:%d %s (%s)\n", __FILE__, __LINE__, #cond,   \
             tamm_last_error());                                  \
      ++fails;                                                    \
    }                                                             \
  } while (0)

int main(void) {
  tamm_space *o = NULL, *v = NULL;
  CHECK(tamm_space_create_spin(3, 2, 2, &o) == TAMM_OK);
  CHECK(tamm_space_create_spin(4, 5, 3, &v) == TAMM_OK);
  int32_t nt = 0;
  int64_t ext = 0;
  CHECK(tamm_space_info(v, &nt, &ext) == TAMM_OK && nt == 4 && ext == 9);

  tamm_space* dv[4] = {v, v, v, v};
  tamm_space* dt[4] = {v, v, o, o};
  tamm_tensor *V = NULL, *T = NULL, *R = NULL;
  CHECK(tamm_tensor_create(dv, 4, NULL, NULL, &V) == TAMM_OK);
  CHECK(tamm_tensor_create(dt, 4, NULL, NULL, &T) == TAMM_OK);
  CHECK(tamm_tensor_create(dt, 4, NULL, NULL, &R) == TAMM_OK);
  int64_t nb = 0;
  CHECK(tamm_tensor_blocks(V, &nb, NULL, NULL) == TAMM_OK && nb > 0);

  tamm_plan* p = NULL;
  CHECK(tamm_plan_create(R, "abij", V, "abcd", T, "cdij", TAMM_PREC_F64, &p) == TAMM_OK);
  tamm_plan_stats st;
  memset(&st, 0, sizeof st);
  CHECK(tamm_plan_stats_get(p, &st) == TAMM_OK && st.tasks > 0 && st.useful_flops > 0.0);
  size_t ws = 0;
  CHECK(tamm_plan_workspace_size(p, &ws) == TAMM_OK && ws >= 256);
  /* executing without bound storage is refused before any GPU work */
  CHECK(tamm_plan_execute(p, 1.0, 0.0, NULL) == TAMM_ERR_UNBOUND);
  CHECK(tamm_plan_destroy(p) == TAMM_OK);

  /* label errors and the one-shot cache's host half */
  CHECK(tamm_plan_create(R, "abij", V, "abcc", T, "cdij", TAMM_PREC_F64, &p) == TAMM_ERR_LABEL);
  CHECK(tamm_contract_cache_clear() == TAMM_OK);
  CHECK(tamm_contract_workspace_size(R, "abij", V, "abcd", T, "cdij", TAMM_PREC_F64, &ws) == TAMM_OK);
  int64_t cached = -1;
  CHECK(tamm_contract_cache_count(&cached) == TAMM_OK && cached == 1);
  CHECK(tamm_contract(R, "abij", V, "abcd", T, "cdij", TAMM_PREC_F64, 1.0, 0.0, NULL, ws, NULL) ==
        TAMM_ERR_WORKSPACE);

  CHECK(tamm_tensor_destroy(R) == TAMM_OK);
  CHECK(tamm_contract_cache_count(&cached) == TAMM_OK && cached == 0);
  CHECK(tamm_tensor_destroy(T) == TAMM_OK && tamm_tensor_destroy(V) == TAMM_OK);
  CHECK(tamm_space_destroy(o) == TAMM_OK && tamm_space_destroy(v) == TAMM_OK);
  printf("%s: tasks %lld, useful flops %.0f, workspace %zu bytes\n", fails ? "FAILED" : "ok", (long long)st.tasks,
         st.useful_flops, ws);
  return fails ? 1 : 0;
}
