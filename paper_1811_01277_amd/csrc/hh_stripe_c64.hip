// One-lane stripe kernel instances for complex fp64 (one translation unit per
// element type, so that the kernel variants compile in parallel).
#include "hh_kernels_impl.h"

namespace ehh {

#define EHH_DIAG(E, DT, NB, K, OCC)                                                    \
  {ELPA_PATH_STRIPE, DT, NB, K, OCC, &launch_diag<E, NB, K, OCC>,                        \
   &launch_diag_batched<E, NB, K, OCC>, &diag_workspace<E, NB, K>}

const StripeEntry* stripe_table_c64(int* size) {
  static const StripeEntry table[] = {
      EHH_DIAG(z64, 2, 32, 4, 2),     EHH_DIAG(z64, 2, 32, 8, 1),
      EHH_DIAG(z64, 2, 64, 2, 1),     EHH_DIAG(z64, 2, 64, 4, 1),
  };
  *size = (int)(sizeof(table) / sizeof(table[0]));
  return table;
}

}  // namespace ehh
