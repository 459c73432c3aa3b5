/* The C ABI used from plain C (compiled with gcc by test_abi.py): the header
 * compiles as C11 and the host-side entry points answer without a GPU. */
#include <stdio.h>
#include <string.h>

#include "trstmi.h"

int main(void) {
  trstmi_params p;
  trstmi_default_params(&p, 4096, 64);
  if (p.n != 4096 || p.d != 64 || p.candidates < 1) return 1;
  p.mode = TRSTMI_MODE_BF16_SCREEN;
  p.candidates = 128;
  if (trstmi_workspace_bytes(&p) == 0) return 2;
  p.n = 1;
  if (trstmi_workspace_bytes(&p) != 0) return 3;
  if (trstmi_coherence(1, 4, TRSTMI_MODE_FP64, NULL, NULL, NULL, 0, NULL) != TRSTMI_E_INVALID_ARG) return 4;
  if (strlen(trstmi_last_error()) == 0) return 5;
  if (trstmi_miso_workspace_bytes(4096, 64, 65536) == 0) return 6;
  if (trstmi_abi_version() < 10) return 7;
  printf("ok\n");
  return 0;
}
