// Table of the compact-WY MFMA kernel instances of every element type
// (hh_wy_r64.hip, hh_wy_r32.hip, hh_wy_c64.hip), concatenated once.
#include <vector>

#include "hh_dispatch.h"

namespace ehh {

const StripeEntry* wy_table_r64(int* size);
const StripeEntry* wy_table_r32(int* size);
const StripeEntry* wy_table_c64(int* size);

const StripeEntry* wy_table(int* size) {
  static const std::vector<StripeEntry> all = [] {
    std::vector<StripeEntry> v;
    for (auto part : {wy_table_r64, wy_table_r32, wy_table_c64}) {
      int c = 0;
      const StripeEntry* t = part(&c);
      v.insert(v.end(), t, t + c);
    }
    return v;
  }();
  *size = (int)all.size();
  return all.data();
}

}  // namespace ehh
