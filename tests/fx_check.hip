// Host-side check of the exact-sum fixed point used by the symmetry merge:
// reads groups of doubles from stdin ("n v1 ... vn" per line), prints the
// sum accumulated as 192-bit fixed point and rounded once, with %a.
#include <cstdio>
#include <vector>

#include "pp_fixed.h"

int main() {
  int n;
  while (std::scanf("%d", &n) == 1) {
    pp::Fx acc{0, 0, 0};
    bool range = false;
    for (int i = 0; i < n; ++i) {
      double v;
      if (std::scanf("%la", &v) != 1) return 2;
      acc = pp::fx_add(acc, pp::fx_from_double(v, &range));
    }
    std::printf("%a %d\n", pp::fx_to_double(acc), range ? 1 : 0);
  }
  return 0;
}
