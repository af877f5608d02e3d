// Host driver for the Golub-Welsch routine shared with the GPU quadrature
// kernel: reads n, diagonal, subdiagonal; prints status, the log quadrature
// and the (eigenvalue, first component) pairs.
#include <cstdio>
#include <vector>

#include "gw_ql.h"

int main() {
  int n = 0;
  if (std::scanf("%d", &n) != 1 || n < 1) return 2;
  std::vector<double> d(n), e(n), z(n);
  for (int i = 0; i < n; ++i)
    if (std::scanf("%lf", &d[i]) != 1) return 2;
  for (int i = 0; i + 1 < n; ++i)
    if (std::scanf("%lf", &e[i]) != 1) return 2;
  const int rc = ld::tridiag_ql_first_row(n, d.data(), e.data(), z.data(), 1);
  int bad = 0;
  const double k = ld::gauss_log_sum(n, d.data(), z.data(), 1, &bad);
  std::printf("%d %d %.17g\n", rc, bad, k);
  for (int i = 0; i < n; ++i) std::printf("%.17g %.17g\n", d[i], z[i]);
  return 0;
}
