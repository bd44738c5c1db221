// Compact-WY MFMA kernel instances for complex fp64 (one translation unit per
// element type, so that the variants compile in parallel).
#include "hh_wy_impl.h"

namespace ehh {

#define EHH_WY(E, DT, NB, K, T, OCC, PF, VP)                                             \
  {ELPA_PATH_WY, DT, NB, K, OCC, &launch_wy<E, NB, K, T, OCC, PF, VP>,                 \
   &launch_wy_batched<E, NB, K, T, OCC, PF, VP>, &wy_workspace<E, NB, K, T>,          \
   &launch_wy_ws<E, NB, K, T, OCC, PF, VP>, nullptr}

const StripeEntry* wy_table_c64(int* size) {
  static const StripeEntry table[] = {
      // planar complex: four real MFMA chains per product
      EHH_WY(z64, 2, 64, 32, 1, 1, false, false), EHH_WY(z64, 2, 64, 48, 1, 1, false, false),
      EHH_WY(z64, 2, 64, 16, 1, 1, true, false),
      EHH_WY(z64, 2, 32, 32, 1, 1, true, false),
  };
  *size = (int)(sizeof(table) / sizeof(table[0]));
  return table;
}

}  // namespace ehh
