/* A plain C99 client of the library: the header compiles as C, the shared
 * library links from C, and the argument checks that run before any device
 * work answer through the C ABI with status codes and messages. */
#include <stdio.h>
#include <string.h>

#include "spdhss.h"

static int fail(const char* what) {
  printf("abi_c_check FAILED: %s (last error: %s)\n", what, spd_last_error());
  return 1;
}

int main(void) {
  double stand_in = 0.0; /* never read: every call below fails its checks first */
  spd_kernel k = {SPD_K_MATERN32, 0.1, 1e-4};
  spd_h2_opts o = {0, 1.0, 1e-8, 8, 128, 2048, 90.0, 1, SPD_TREE_KD}; /* leaf_size 0 is invalid */
  spd_h2_t h = (spd_h2_t)&stand_in;
  if (h2_build(&stand_in, 100, k, &o, NULL, &h) != SPD_E_INVALID) return fail("h2_build status");
  if (h != NULL) return fail("h2_build clears *out");
  if (strstr(spd_last_error(), "leaf_size") == NULL) return fail("h2_build message");

  o.leaf_size = 64;
  o.tree = 2;
  if (h2_build(&stand_in, 100, k, &o, NULL, &h) != SPD_E_INVALID) return fail("unknown tree kind");
  o.tree = SPD_TREE_BOX;
  k.ell = -1.0;
  if (h2_build(&stand_in, 100, k, &o, NULL, &h) != SPD_E_INVALID) return fail("negative ell");

  spd_hss_t m = NULL;
  if (spdhss_build(NULL, NULL, NULL, &m) != SPD_E_INVALID || m != NULL) return fail("spdhss_build");
  if (pcg_solve(NULL, NULL, &stand_in, &stand_in, 1, 1, 1e-8, 10, NULL, NULL, NULL) != SPD_E_INVALID)
    return fail("pcg_solve");

  spd_server_t srv = NULL;
  if (spd_server_create(0, 1, &srv) != SPD_E_INVALID || srv != NULL) return fail("spd_server_create");
  if (spd_request_footprint(NULL) != 0) return fail("spd_request_footprint");

  h2_destroy(NULL);
  spdhss_destroy(NULL);
  ulv_destroy(NULL);
  printf("abi_c_check ok\n");
  return 0;
}
