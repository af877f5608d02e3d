// Host driver for the Hessenberg-log routine shared with the GPU kernel:
// reads n and H (n x n, row-major); prints the status and log(H) e1.  The
// Gauss-Legendre nodes on [0, 1] come from the Golub-Welsch routine applied
// to the Legendre Jacobi matrix, as in the library.
#include <cmath>
#include <cstdio>
#include <vector>

#include "gw_ql.h"
#include "hess_log.h"

int main() {
  int n = 0;
  if (std::scanf("%d", &n) != 1 || n < 1) return 2;
  std::vector<double> H((size_t)n * n);
  for (auto& x : H)
    if (std::scanf("%lf", &x) != 1) return 2;
  const int q = ld::kLogNodes;
  std::vector<double> d(q, 0.0), e(q, 0.0), z(q);
  for (int j = 1; j < q; ++j) e[j - 1] = j / std::sqrt(4.0 * j * j - 1.0);
  ld::tridiag_ql_first_row(q, d.data(), e.data(), z.data(), 1);
  std::vector<double> nodes(q), weights(q);
  for (int j = 0; j < q; ++j) {
    nodes[j] = 0.5 * (d[j] + 1.0);
    weights[j] = z[j] * z[j];
  }
  std::vector<double> ell(n), ws(ld::hess_log_workspace(n));
  std::vector<double> shd(8);
  std::vector<int> shi(8);
  ld::TeamScratch sc{shd.data(), shi.data()};
  ld::HostTeam tm;
  const int rc = ld::team_hess_log_e1(tm, n, H.data(), n, ell.data(), ws.data(), sc, nodes.data(),
                                      weights.data());
  std::printf("%d\n", rc);
  for (int i = 0; i < n; ++i) std::printf("%.17g\n", ell[i]);
  return 0;
}
