/* Host-only use of the C ABI from plain C: a two-tensor network of two
 * qubits sharing one bond, a = sum_b T0[x0][b] T1[x1][b], planned for all
 * four bitstrings.  Prints the plan figures and exercises one error path;
 * no device call is made. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "matnc.h"

int main(void) {
  /* index ids: 0 = output of qubit 0, 1 = output of qubit 1, 2 = bond */
  const int ranks[2] = {2, 2};
  const int ids[4] = {0, 2, 1, 2};
  double data[2 * 8];
  for (int i = 0; i < 16; ++i) data[i] = 0.25 * (i + 1);
  const int out_index[2] = {0, 1};
  matnc_network net = NULL;
  if (matnc_network_create(2, ranks, ids, data, 2, out_index, &net) != MATNC_OK) {
    printf("network_create failed: %s\n", matnc_last_error());
    return 1;
  }
  const int pairs[2] = {0, 1};
  const uint64_t words[4] = {0, 1, 2, 3};
  matnc_plan plan = NULL;
  if (matnc_plan_create(net, pairs, 0, NULL, 0, NULL, 4, words, MATNC_C64, 32, 1, 0, &plan) != MATNC_OK) {
    printf("plan_create failed: %s\n", matnc_last_error());
    return 1;
  }
  matnc_plan_info_t info;
  memset(&info, 0, sizeof info);
  if (matnc_plan_info(plan, &info) != MATNC_OK) return 1;
  printf("version %s\n", matnc_version());
  printf("n_amplitudes %lld n_unique %lld n_slices %lld n_nodes %d max_rank %d\n", (long long)info.n_amplitudes,
         (long long)info.n_unique, (long long)info.n_slices, info.n_nodes, info.max_rank);
  printf("cmac_single %.1f cmac_multi %.1f workspace_bytes %zu\n", info.cmac_single, info.cmac_multi,
         info.workspace_bytes);
  /* a tree that uses tensor 0 twice is rejected with a message */
  const int bad[2] = {0, 0};
  matnc_plan p2 = NULL;
  const int rc = matnc_plan_create(net, bad, 0, NULL, 0, NULL, 4, words, MATNC_C64, 32, 1, 0, &p2);
  printf("bad tree rc %d (%s) message %s\n", rc, rc == MATNC_E_INVALID ? "invalid" : "?",
         strlen(matnc_last_error()) > 0 ? "present" : "missing");
  /* execute before bind is an ordering error */
  printf("execute before bind rc %d\n", matnc_execute(plan, 0, 1, NULL));
  matnc_plan_destroy(plan);
  matnc_network_destroy(net);
  return 0;
}
