// Two-lane stripe kernel instances for real fp32 (one translation unit per
// element type, so that the kernel variants compile in parallel).
#include "hh_split_impl.h"

namespace ehh {

#define EHH_SPLIT(E, DT, NB, K, OCC, PD)                                               \
  {ELPA_PATH_SPLIT, DT, NB, K, OCC, &launch_split<E, NB, K, OCC, PD>,              \
   &launch_split_batched<E, NB, K, OCC, PD>, &split_workspace<E, NB, K>,           \
   &launch_split_ws<E, NB, K, OCC, PD>, &prepare_split<E, NB, K, OCC, PD>}

const StripeEntry* split_table_r32(int* size) {
  static const StripeEntry table[] = {
      // one register per value, up to four waves per SIMD
      EHH_SPLIT(float, 1, 64, 64, 4, 2), EHH_SPLIT(float, 1, 64, 80, 4, 2),
      EHH_SPLIT(float, 1, 64, 96, 4, 1),
      EHH_SPLIT(float, 1, 32, 64, 4, 2), EHH_SPLIT(float, 1, 32, 96, 4, 2),
      EHH_SPLIT(float, 1, 32, 128, 3, 1),
  };
  *size = (int)(sizeof(table) / sizeof(table[0]));
  return table;
}

}  // namespace ehh
