// Golub-Welsch reduction of a symmetric tridiagonal matrix, shared by the
// GPU quadrature kernel and a host unit test.
//
// Gauss quadrature from Lanczos (Section 3.1, eq. gauss_quadrature): for the
// m x m tridiagonal T_m of a unit start vector, v^T f(Q) v is approximated by
// sum_k tau_k^2 f(theta_k), with theta_k the eigenvalues of T_m and tau_k the
// first component of the k-th unit eigenvector.  Only the first row of the
// eigenvector matrix is needed, so the implicit QL iteration below applies
// each plane rotation to that row alone (Golub & Welsch, Math. Comp. 1969):
// O(m^2) work instead of O(m^3).
//
// The iteration is the implicitly shifted QL algorithm for symmetric
// tridiagonal matrices in the form published by Bowdler, Martin, Reinsch and
// Wilkinson ("The QR and QL algorithms for symmetric matrices", Numer. Math.
// 11, 1968; the procedure later distributed as EISPACK's imtql2): deflate
// when |e_i| <= eps (|d_i|+|d_i+1|), otherwise take the Wilkinson-type shift
// from the eigenvalue of the leading 2x2 block closest to d_l and chase the
// bulge upward with Givens rotations.  Golub and Welsch's contribution used
// here is to carry only the first row of the rotations.
#pragma once

#include <math.h>
#include <float.h>

#ifndef LD_HD
#if defined(__HIPCC__)
#define LD_HD __host__ __device__
#else
#define LD_HD
#endif
#endif

namespace ld {

// d[i*stride] (i < n): diagonal, overwritten by the eigenvalues.
// e[i*stride] (i < n-1): subdiagonal; e[(n-1)*stride] is scratch.
// z[i*stride]: on entry anything, on exit the first eigenvector components.
// Optional rotation log (rot_c, rot_s, rot_i non-null, capacity rot_cap):
// every plane rotation applied to the eigenvector columns (i, i+1) is
// appended in order, so that U y = G_1 (G_2 (... G_N y)) can be replayed;
// *rot_n receives the count (-1 when the capacity was exceeded).
// Returns 0 on success, 1 when an eigenvalue needed more than 64 sweeps.
LD_HD inline int tridiag_ql_first_row(int n, double* d, double* e, double* z, int stride,
                                      double* rot_c = nullptr, double* rot_s = nullptr,
                                      int* rot_i = nullptr, int rot_cap = 0,
                                      int* rot_n = nullptr) {
  int nrot = 0;
#define LD_D(i) d[(i) * stride]
#define LD_E(i) e[(i) * stride]
#define LD_Z(i) z[(i) * stride]
  for (int i = 0; i < n; ++i) LD_Z(i) = (i == 0) ? 1.0 : 0.0;
  if (n > 0) LD_E(n - 1) = 0.0;
  for (int l = 0; l < n; ++l) {
    for (int sweep = 0;; ++sweep) {
      int mm = l;
      for (; mm < n - 1; ++mm) {
        const double dd = fabs(LD_D(mm)) + fabs(LD_D(mm + 1));
        if (fabs(LD_E(mm)) <= DBL_EPSILON * dd) break;
      }
      if (mm == l) break;  // d_l has converged
      if (sweep == 64) {
        if (rot_n) *rot_n = -1;
        return 1;
      }
      // shift: eigenvalue of [[d_l, e_l], [e_l, d_l+1]] nearest d_l, expressed
      // relative to d_mm so that the chase starts from the bottom of the block
      double g = (LD_D(l + 1) - LD_D(l)) / (2.0 * LD_E(l));
      double r = hypot(g, 1.0);
      g = LD_D(mm) - LD_D(l) + LD_E(l) / (g + copysign(r, g));
      double s = 1.0, c = 1.0, p = 0.0;
      bool split = false;
      for (int i = mm - 1; i >= l; --i) {
        const double f = s * LD_E(i);
        const double b = c * LD_E(i);
        r = hypot(f, g);
        LD_E(i + 1) = r;
        if (r == 0.0) {  // an off-diagonal vanished: the block splits
          LD_D(i + 1) -= p;
          LD_E(mm) = 0.0;
          split = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = LD_D(i + 1) - p;
        r = (LD_D(i) - g) * s + 2.0 * c * b;
        p = s * r;
        LD_D(i + 1) = g + p;
        g = c * r - b;
        const double zi1 = LD_Z(i + 1);
        LD_Z(i + 1) = s * LD_Z(i) + c * zi1;
        LD_Z(i) = c * LD_Z(i) - s * zi1;
        if (rot_c) {
          if (nrot < rot_cap) {
            rot_c[nrot] = c;
            rot_s[nrot] = s;
            rot_i[nrot] = i;
          }
          ++nrot;
        }
      }
      if (split) continue;
      LD_D(l) -= p;
      LD_E(l) = g;
      LD_E(mm) = 0.0;
    }
  }
  if (rot_n) *rot_n = (nrot <= rot_cap) ? nrot : -1;
  return 0;
#undef LD_D
#undef LD_E
#undef LD_Z
}

// sum_k z_k^2 log(theta_k) after tridiag_ql_first_row; *bad is set when a
// Ritz value is not positive (the operator is then not SPD).
LD_HD inline double gauss_log_sum(int n, const double* d, const double* z, int stride, int* bad) {
  double acc = 0.0;
  for (int k = 0; k < n; ++k) {
    const double th = d[k * stride];
    const double w = z[k * stride] * z[k * stride];
    if (!(th > 0.0)) {
      *bad = 1;
      continue;
    }
    acc += w * log(th);
  }
  return acc;
}

// y <- U y for U = G_1 G_2 ... G_N, the rotations logged by
// tridiag_ql_first_row (G_q acts on entries (i, i+1): y_i' = c y_i + s y_i+1,
// y_i+1' = c y_i+1 - s y_i), applied last one first.
LD_HD inline void apply_logged_rotations(int nrot, const double* rot_c, const double* rot_s,
                                         const int* rot_i, double* y, int stride) {
  for (int q = nrot - 1; q >= 0; --q) {
    const int i = rot_i[q];
    const double c = rot_c[q], s = rot_s[q];
    const double a = y[i * stride], b = y[(i + 1) * stride];
    y[i * stride] = c * a + s * b;
    y[(i + 1) * stride] = c * b - s * a;
  }
}

}  // namespace ld
