// One-lane stripe kernel instances for real fp64 (one translation unit per
// element type, so that the kernel variants compile in parallel).
#include "hh_kernels_impl.h"

namespace ehh {

#define EHH_DIAG(E, DT, NB, K, OCC)                                                    \
  {ELPA_PATH_STRIPE, DT, NB, K, OCC, &launch_diag<E, NB, K, OCC>,                        \
   &launch_diag_batched<E, NB, K, OCC>, &diag_workspace<E, NB, K>}

const StripeEntry* stripe_table_r64(int* size) {
  static const StripeEntry table[] = {
      EHH_DIAG(double, 0, 32, 8, 2),  EHH_DIAG(double, 0, 32, 16, 2),
      EHH_DIAG(double, 0, 32, 32, 2), EHH_DIAG(double, 0, 32, 48, 1),
      EHH_DIAG(double, 0, 64, 8, 2),  EHH_DIAG(double, 0, 64, 16, 2),
      EHH_DIAG(double, 0, 64, 24, 2), EHH_DIAG(double, 0, 64, 32, 2),
      EHH_DIAG(double, 0, 64, 40, 1), EHH_DIAG(double, 0, 64, 48, 1),
  };
  *size = (int)(sizeof(table) / sizeof(table[0]));
  return table;
}

}  // namespace ehh
