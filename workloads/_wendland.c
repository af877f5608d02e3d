/* Neighbour search and CSR assembly of the Wendland C2 covariance on points
 * sorted by square cells of side 1/ncell >= rho (seeded input generation;
 * none of the estimator's arithmetic).
 *
 * Points are given in cell order (cell id cy * ncell + cx ascending, and in
 * ascending index within a cell), with cell_start[c] .. cell_start[c+1]-1 the
 * indices of cell c.  Every pair at distance below rho lies in the 3 x 3
 * block of cells around a point, and visiting those cells in ascending id
 * lists each row's columns in ascending order.  Per pair the arithmetic is
 * the one the NumPy generator uses, in the same order and without fused
 * multiply-adds (compile with -ffp-contract=off): d = p_min - p_max,
 * r = sqrt(dx*dx + dy*dy) / rho, kept when r < 1, value
 * scale * ((1 - r)^2)^2 * (4 r + 1) (only correctly rounded operations, so
 * both sides agree bit for bit); the diagonal is scale + nugget.
 */
#include <math.h>
#include <stdint.h>

static double wendland_r(const double* p, int64_t i, int64_t j, double rho) {
  const int64_t a = i < j ? i : j, b = i < j ? j : i;
  const double dx = p[2 * a] - p[2 * b];
  const double dy = p[2 * a + 1] - p[2 * b + 1];
  return sqrt(dx * dx + dy * dy) / rho;
}

/* counts[i] = entries of row i (diagonal included) for rows [r0, r1). */
void wendland_count(int64_t r0, int64_t r1, const double* pts, const int64_t* cell_of,
                    const int64_t* cell_start, int64_t ncell, double rho, int64_t* counts) {
  for (int64_t i = r0; i < r1; ++i) {
    const int64_t c = cell_of[i], cy = c / ncell, cx = c % ncell;
    int64_t cnt = 0;
    for (int64_t y = cy - 1; y <= cy + 1; ++y) {
      if (y < 0 || y >= ncell) continue;
      for (int64_t x = cx - 1; x <= cx + 1; ++x) {
        if (x < 0 || x >= ncell) continue;
        const int64_t cc = y * ncell + x;
        for (int64_t j = cell_start[cc]; j < cell_start[cc + 1]; ++j)
          if (j == i || wendland_r(pts, i, j, rho) < 1.0) ++cnt;
      }
    }
    counts[i] = cnt;
  }
}

/* Columns and values of rows [r0, r1) at row_ptr[i] onwards. */
void wendland_fill(int64_t r0, int64_t r1, const double* pts, const int64_t* cell_of,
                   const int64_t* cell_start, int64_t ncell, double rho, double scale,
                   double nugget, const int64_t* row_ptr, int32_t* col, double* val) {
  for (int64_t i = r0; i < r1; ++i) {
    const int64_t c = cell_of[i], cy = c / ncell, cx = c % ncell;
    int64_t k = row_ptr[i];
    for (int64_t y = cy - 1; y <= cy + 1; ++y) {
      if (y < 0 || y >= ncell) continue;
      for (int64_t x = cx - 1; x <= cx + 1; ++x) {
        if (x < 0 || x >= ncell) continue;
        const int64_t cc = y * ncell + x;
        for (int64_t j = cell_start[cc]; j < cell_start[cc + 1]; ++j) {
          if (j == i) {
            col[k] = (int32_t)j;
            val[k++] = scale + nugget;
            continue;
          }
          const double r = wendland_r(pts, i, j, rho);
          if (r < 1.0) {
            col[k] = (int32_t)j;
            const double t = 1.0 - r, t2 = t * t;
            val[k++] = scale * (t2 * t2) * (4.0 * r + 1.0);
          }
        }
      }
    }
  }
}
