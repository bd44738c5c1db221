// Compact-WY MFMA kernel instances for real fp32 (one translation unit per
// element type, so that the variants compile in parallel).
#include "hh_wy_impl.h"

namespace ehh {

#define EHH_WY(E, DT, NB, K, T, OCC, PF, VP)                                             \
  {ELPA_PATH_WY, DT, NB, K, OCC, &launch_wy<E, NB, K, T, OCC, PF, VP>,                 \
   &launch_wy_batched<E, NB, K, T, OCC, PF, VP>, &wy_workspace<E, NB, K, T>,          \
   &launch_wy_ws<E, NB, K, T, OCC, PF, VP>, nullptr}

const StripeEntry* wy_table_r32(int* size) {
  static const StripeEntry table[] = {
      EHH_WY(float, 1, 64, 64, 2, 2, true, false), EHH_WY(float, 1, 64, 96, 2, 1, true, true),
      EHH_WY(float, 1, 64, 128, 2, 1, true, true), EHH_WY(float, 1, 64, 32, 2, 2, true, false),
      EHH_WY(float, 1, 64, 160, 2, 1, true, true), EHH_WY(float, 1, 64, 192, 2, 1, true, true),
      EHH_WY(float, 1, 32, 64, 4, 1, true, true), EHH_WY(float, 1, 32, 96, 2, 1, true, true),
  };
  *size = (int)(sizeof(table) / sizeof(table[0]));
  return table;
}

}  // namespace ehh
