// Matrix-core axis pass (FP64 instantiation) and the host code that writes the
// split-product fragment tables of D and D^T into the plan.
#include <vector>

#include "cheb_host.h"
#include "dense_launch.h"

namespace cheb {

template int launch_dense_batch<double>(const cheb_plan*, int, int, const double*, const double*, double*, const DenseSys*,
                                      const int*, int, hipStream_t);
template int launch_dense_pass<double>(const cheb_plan*, int, int, int, const double*, const double*, double*,
                                       const double*, hipStream_t);
template int launch_dense_pair<double>(const cheb_plan*, int, const double*, const double*, double*, double*, hipStream_t);
template bool dense_pair_ok<double>(const cheb_plan*);
template int launch_dense_dacc<double>(const cheb_plan*, int, const double*, const double*, double*, hipStream_t);
template int launch_dense_jac<double>(const cheb_plan*, const double*, const double* const*, const double*, double*,
                                      hipStream_t);

// Ao / Ae / middle-row fragment table of a centro-antisymmetric n x n matrix M
// (row-major), in the lane order the kernel loads: entry (mt, ks, lane) holds
// the operand of row 16 mt + lane % 16 and column 4 ks + lane / 16.
static void dense_table(int N, const std::vector<double>& M, double* tab) {
  const DenseDims S = dense_dims(N);
  const int n = N + 1;
  for (int i = 0; i < S.TAB; ++i) tab[i] = 0.0;
  auto m = [&](int i, int j) { return M[(size_t)i * n + j]; };
  auto ao = [&](int i, int j) { return 0.5 * (m(i, j) - m(i, N - j)); };
  auto ae = [&](int i, int j) { return (S.EVEN && 2 * j == N) ? 0.5 * m(i, j) : 0.5 * (m(i, j) + m(i, N - j)); };
  for (int mt = 0; mt < S.MT; ++mt)
    for (int l = 0; l < 64; ++l) {
      const int i = 16 * mt + (l & 15);
      if (i >= S.RM) continue;
      for (int ks = 0; ks < S.KO4; ++ks) {
        const int j = 4 * ks + (l >> 4);
        if (j < S.KO) tab[(mt * S.KO4 + ks) * 64 + l] = ao(i, j);
      }
      for (int ks = 0; ks < S.KE4; ++ks) {
        const int j = 4 * ks + (l >> 4);
        if (j < S.KE) tab[S.OFF_E + (mt * S.KE4 + ks) * 64 + l] = ae(i, j);
      }
    }
  if (S.MIDV)
    for (int j = 0; j < S.KO; ++j) tab[S.OFF_MID + j] = ao(S.HALF, j);
  for (int i = 0; i < n; ++i) {
    tab[S.OFF_COL + i] = m(i, 0);
    tab[S.OFF_COL + n + i] = m(i, N);
  }
}

int dense_setup(cheb_plan* p) {
  size_t total = 0;
  for (int a = 0; a < 3; ++a) {
    p->dd_ok[a] = dense_supported(p->ax[a].N) ? 1 : 0;
    // default tile shape (measured on MI355X): the 4-wave register-fragment
    // tiles, faster than the 8-wave LDS-table tiles at every N in both
    // precisions (FP32 at N = 128: 35.8 against 40.9 us per apply);
    // cheb_plan_autotune replaces it by timing
    p->dense_var[a][0] = 1;
    p->dense_var[a][1] = 1;
    for (int t = 0; t < 2; ++t) {
      p->dd_off[a][t] = total;
      if (p->dd_ok[a]) total += round_up((size_t)dense_dims(p->ax[a].N).TAB, 64);
    }
  }
  p->dd64 = nullptr;
  p->dd32 = nullptr;
  if (total == 0) return CHEB_OK;
  std::vector<double> h(total, 0.0);
  for (int a = 0; a < 3; ++a) {
    if (!p->dd_ok[a]) continue;
    const int N = p->ax[a].N, n = N + 1;
    std::vector<double> D, Dt((size_t)n * n);
    dense_D(N, p->ax[a].L, D);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) Dt[(size_t)i * n + j] = D[(size_t)j * n + i];
    dense_table(N, D, h.data() + p->dd_off[a][0]);
    dense_table(N, Dt, h.data() + p->dd_off[a][1]);
  }
  std::vector<float> h32(total);
  for (size_t i = 0; i < total; ++i) h32[i] = float(h[i]);
  int rc = hip_check(hipMalloc((void**)&p->dd64, total * sizeof(double)), "hipMalloc(matrix-core tables)");
  if (!rc) rc = hip_check(hipMalloc((void**)&p->dd32, total * sizeof(float)), "hipMalloc(matrix-core tables)");
  if (!rc)
    rc = hip_check(hipMemcpy(p->dd64, h.data(), total * sizeof(double), hipMemcpyHostToDevice),
                   "hipMemcpy(matrix-core tables)");
  if (!rc)
    rc = hip_check(hipMemcpy(p->dd32, h32.data(), total * sizeof(float), hipMemcpyHostToDevice),
                   "hipMemcpy(matrix-core tables)");
  // second output of the two-axis launch (x and y passes together), for plans
  // whose three axes can all take the matrix-core route with equal N on x, y;
  // optional: without it an apply takes three launches
  if (!rc && p->dd_ok[0] && p->dd_ok[1] && p->dd_ok[2] && p->ax[0].N == p->ax[1].N) {
    const size_t bytes = p->npts * (p->prec == CHEB_F32 ? sizeof(float) : sizeof(double));
    if (hipMalloc(&p->pair_buf, bytes) != hipSuccess) {
      (void)hipGetLastError();
      p->pair_buf = nullptr;
    }
  }
  return rc;
}

}  // namespace cheb
