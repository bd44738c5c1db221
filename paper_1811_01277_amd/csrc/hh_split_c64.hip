// Two-lane stripe kernel instances for complex fp64 (one translation unit per
// element type, so that the kernel variants compile in parallel).
#include "hh_split_impl.h"

namespace ehh {

#define EHH_SPLIT(E, DT, NB, K, OCC, PD)                                               \
  {ELPA_PATH_SPLIT, DT, NB, K, OCC, &launch_split<E, NB, K, OCC, PD>,              \
   &launch_split_batched<E, NB, K, OCC, PD>, &split_workspace<E, NB, K>,           \
   &launch_split_ws<E, NB, K, OCC, PD>, &prepare_split<E, NB, K, OCC, PD>}

const StripeEntry* split_table_c64(int* size) {
  static const StripeEntry table[] = {
      // each window register holds two fp64 values
      EHH_SPLIT(z64, 2, 64, 16, 2, 2), EHH_SPLIT(z64, 2, 64, 24, 2, 1),
      EHH_SPLIT(z64, 2, 32, 32, 2, 2), EHH_SPLIT(z64, 2, 32, 48, 2, 1),
  };
  *size = (int)(sizeof(table) / sizeof(table[0]));
  return table;
}

}  // namespace ehh
