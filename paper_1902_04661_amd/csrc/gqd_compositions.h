// Placeholder until the derived table is generated.
#pragma once
namespace gqd {
struct FlatComp {
  int order;
  int count;
  int offset;
};
constexpr int kNumFlat = 1;
constexpr FlatComp kFlatComps[kNumFlat] = {{2, 1, 0}};
constexpr int kFlatTauLen = 1;
#define GQD_FLAT_TAU_VALUES 1.0
}  // namespace gqd
