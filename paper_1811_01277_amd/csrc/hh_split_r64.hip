// Two-lane stripe kernel instances for real fp64 (one translation unit per
// element type, so that the kernel variants compile in parallel).
#include "hh_split_impl.h"

namespace ehh {

#define EHH_SPLIT(E, DT, NB, K, OCC, PD)                                               \
  {ELPA_PATH_SPLIT, DT, NB, K, OCC, &launch_split<E, NB, K, OCC, PD>,              \
   &launch_split_batched<E, NB, K, OCC, PD>, &split_workspace<E, NB, K>,           \
   &launch_split_ws<E, NB, K, OCC, PD>, &prepare_split<E, NB, K, OCC, PD>}

const StripeEntry* split_table_r64(int* size) {
  static const StripeEntry table[] = {
      EHH_SPLIT(double, 0, 32, 32, 2, 1), EHH_SPLIT(double, 0, 32, 64, 2, 1),
      EHH_SPLIT(double, 0, 32, 96, 2, 1),
      // reflector pairs, the last number the pairs whose values are in
      // flight; k = 48 and 64 fit three waves per SIMD, k = 80 two
      EHH_SPLIT(double, 0, 64, 48, 2, 1), EHH_SPLIT(double, 0, 64, 64, 2, 1),
      EHH_SPLIT(double, 0, 64, 80, 2, 2),
  };
  *size = (int)(sizeof(table) / sizeof(table[0]));
  return table;
}

}  // namespace ehh
