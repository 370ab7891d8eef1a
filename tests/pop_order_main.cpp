// Prints the sweep pop order of wts_order.h for pair sets read from stdin:
//   n reverse / n column counts / n strip counts   ->   one "q s" line per strip.
#include <cstdio>
#include <vector>

#include "wts_order.h"

int main() {
  int n = 0, reverse = 0;
  if (std::scanf("%d %d", &n, &reverse) != 2 || n < 0) return 2;
  std::vector<long long> c(n);
  std::vector<int64_t> cols(n);
  std::vector<int> strips(n);
  for (int q = 0; q < n; ++q) {
    if (std::scanf("%lld", &c[q]) != 1) return 2;
    cols[q] = c[q];
  }
  for (int q = 0; q < n; ++q)
    if (std::scanf("%d", &strips[q]) != 1) return 2;
  wts::pop_order(cols, strips, reverse != 0, [](int q, int s) { std::printf("%d %d\n", q, s); });
  return 0;
}
