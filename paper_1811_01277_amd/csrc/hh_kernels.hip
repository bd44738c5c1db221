// Reference kernel launchers and the table of the one-lane stripe kernel
// instances of every element type (hh_stripe_r64.hip, hh_stripe_r32.hip,
// hh_stripe_c64.hip), concatenated once.
#include <vector>

#include "hh_kernels_impl.h"

namespace ehh {

const StripeEntry* stripe_table_r64(int* size);
const StripeEntry* stripe_table_r32(int* size);
const StripeEntry* stripe_table_c64(int* size);

const StripeEntry* stripe_table(int* size) {
  static const std::vector<StripeEntry> all = [] {
    std::vector<StripeEntry> v;
    for (auto part : {stripe_table_r64, stripe_table_r32, stripe_table_c64}) {
      int c = 0;
      const StripeEntry* t = part(&c);
      v.insert(v.end(), t, t + c);
    }
    return v;
  }();
  *size = (int)all.size();
  return all.data();
}

RefLaunch ref_launcher(int dtype) {
  switch (dtype) {
    case 0: return &launch_ref<double>;
    case 1: return &launch_ref<float>;
    case 2: return &launch_ref<z64>;
    default: return nullptr;
  }
}

}  // namespace ehh
