// Table of the two-lane stripe kernel instances of every element type
// (hh_split_r64.hip, hh_split_r32.hip, hh_split_c64.hip), concatenated once.
#include <vector>

#include "hh_dispatch.h"

namespace ehh {

const StripeEntry* split_table_r64(int* size);
const StripeEntry* split_table_r32(int* size);
const StripeEntry* split_table_c64(int* size);

const StripeEntry* split_table(int* size) {
  static const std::vector<StripeEntry> all = [] {
    std::vector<StripeEntry> v;
    for (auto part : {split_table_r64, split_table_r32, split_table_c64}) {
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
