// Fast-diagonalisation preconditioner for the reduced collocation operator
// (an extension: the paper's solver is unpreconditioned LGMRES).
//
// For a constant conductivity Kc the reduced operator is the Kronecker sum
// Kc (A_x (+) A_y (+) A_z) of the 1-D reduced operators A_a = R D_a D_a L_a
// (second derivative on the interior nodes of one pencil, end values lifted by
// that axis' boundary rows).  With A_a = V_a diag(lambda_a) V_a^{-1},
//   M^{-1} = (V_x (x) V_y (x) V_z) diag(1 / (Kc (lx_i + ly_j + lz_k))) (V_x^{-1} (x) ...),
// the exact inverse for constant K and a spectrally close one for variable K
// (Kc = mean of K).  Right preconditioning leaves the discrete solution unchanged.
//
// Setup (host, once per plan): the 1-D matrices from the closed-form
// differentiation matrix, a real nonsymmetric eigensolver (Householder
// reduction to Hessenberg form, implicit single-shift QR with Wilkinson shifts
// to the real Schur form -- the eigenvalues of these operators are real -- and
// back-substitution for the eigenvectors), and the inverse by Gauss-Jordan.
// An axis with the same face type at both ends has a centro-symmetric 1-D
// operator, which splits into two half-size problems.
// Apply (device): pack interior -> three dense axis contractions with V^{-1}
// -> divide by the eigenvalue sums -> three contractions with V -> unpack (for
// m <= 128 the packing, scaling and unpacking run inside the contractions).
// The contractions run on the matrix cores (MFMA 16x16x4): a pencil-tile kernel
// for m <= 128, a generic strided batched GEMM beyond.
#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

#include "cheb_host.h"
#include "dev_common.h"
#include "internal.h"

namespace cheb {

// ---------------------------------------------------------------------------
// host linear algebra
// ---------------------------------------------------------------------------
namespace {

// 1-D reduced operator R D D L (m x m, m = N-1) for the boundary pair (blo, bhi)
// with Robin coefficients (slo, shi) on Neumann ends
void reduced_1d(int N, double L, int blo, int bhi, double slo, double shi, std::vector<double>& A) {
  const int n = N + 1, m = N - 1;
  std::vector<double> D;
  dense_D(N, L, D);
  // lift: rows 0 and N of L as functions of the interior values; the end-value
  // block of the rows -(D u)_0 + slo u_0 and (D u)_N + shi u_N
  std::vector<double> l0(m, 0.0), lN(m, 0.0);
  const double d00 = D[0] - slo, d0N = D[N], dN0 = D[(size_t)N * n], dNN = D[(size_t)N * n + N] + shi;
  for (int j = 0; j < m; ++j) {
    const double a = D[j + 1], b = D[(size_t)N * n + j + 1];
    if (blo == 1 && bhi == 1) {
      const double det = d00 * dNN - d0N * dN0;
      l0[j] = -(dNN * a - d0N * b) / det;
      lN[j] = -(d00 * b - dN0 * a) / det;
    } else if (blo == 1) {
      l0[j] = -a / d00;
    } else if (bhi == 1) {
      lN[j] = -b / dNN;
    }
  }
  // DD on the interior rows 1..N-1 (the only ones A uses), k ascending per entry
  std::vector<double> D2((size_t)n * n, 0.0);
  const double* __restrict__ Dp = D.data();
  for (int i = 1; i < N; ++i) {
    double* __restrict__ row = D2.data() + (size_t)i * n;
    for (int k = 0; k < n; ++k) {
      const double dik = Dp[(size_t)i * n + k];
      if (dik == 0.0) continue;
      const double* __restrict__ dk = Dp + (size_t)k * n;
      for (int j = 0; j < n; ++j) row[j] += dik * dk[j];
    }
  }
  A.assign((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j)
      A[(size_t)i * m + j] = D2[(size_t)(i + 1) * n + (j + 1)] + D2[(size_t)(i + 1) * n] * l0[j] +
                             D2[(size_t)(i + 1) * n + N] * lN[j];
}

// Real nonsymmetric eigen-decomposition for matrices with real eigenvalues.
// A (m x m row-major) is destroyed.  On success V holds unit eigenvectors as
// columns and lam the eigenvalues; returns false if the QR iteration failed.
bool eig_real(int m, std::vector<double>& A, std::vector<double>& lam, std::vector<double>& V) {
  auto H = [&](int i, int j) -> double& { return A[(size_t)i * m + j]; };
  // accumulated orthogonal transform, stored transposed (row k of Zt is
  // column k of Z) so that its updates run along contiguous rows
  std::vector<double> Zt((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) Zt[(size_t)i * m + i] = 1.0;
  auto Zr = [&](int k) { return &Zt[(size_t)k * m]; };
  std::vector<double> zs(m);
  // Householder reduction to upper Hessenberg form, accumulating Z
  std::vector<double> v(m);
  for (int k = 0; k + 2 < m; ++k) {
    double alpha = 0.0;
    for (int i = k + 1; i < m; ++i) alpha += H(i, k) * H(i, k);
    alpha = std::sqrt(alpha);
    if (alpha == 0.0) continue;
    if (H(k + 1, k) > 0) alpha = -alpha;
    for (int i = 0; i < m; ++i) v[i] = 0.0;
    v[k + 1] = H(k + 1, k) - alpha;
    for (int i = k + 2; i < m; ++i) v[i] = H(i, k);
    double vn = 0.0;
    for (int i = k + 1; i < m; ++i) vn += v[i] * v[i];
    if (vn == 0.0) continue;
    // H = P H P, P = I - 2 v v^T / vn; the left product row by row:
    // zs_j = sum_i v_i H(i, j) (i ascending), then H(i, j) -= (2/vn) v_i zs_j
    std::fill(zs.begin(), zs.end(), 0.0);
    for (int i = k + 1; i < m; ++i) {
      const double vi = v[i];
      const double* hr = &H(i, 0);
      for (int j = 0; j < m; ++j) zs[j] += vi * hr[j];
    }
    for (int j = 0; j < m; ++j) zs[j] *= 2.0 / vn;
    for (int i = k + 1; i < m; ++i) {
      const double vi = v[i];
      double* hr = &H(i, 0);
      for (int j = 0; j < m; ++j) hr[j] -= zs[j] * vi;
    }
    for (int i = 0; i < m; ++i) {
      double s = 0.0;
      for (int j = k + 1; j < m; ++j) s += H(i, j) * v[j];
      s *= 2.0 / vn;
      for (int j = k + 1; j < m; ++j) H(i, j) -= s * v[j];
    }
    // Z = Z P: zs_i = sum_j Z(i,j) v_j (j ascending), then Z(i,j) -= (2/vn) zs_i v_j
    std::fill(zs.begin(), zs.end(), 0.0);
    for (int j = k + 1; j < m; ++j) {
      const double vj = v[j];
      const double* zr = Zr(j);
      for (int i = 0; i < m; ++i) zs[i] += zr[i] * vj;
    }
    for (int i = 0; i < m; ++i) zs[i] *= 2.0 / vn;
    for (int j = k + 1; j < m; ++j) {
      const double vj = v[j];
      double* zr = Zr(j);
      for (int i = 0; i < m; ++i) zr[i] -= zs[i] * vj;
    }
    for (int i = k + 2; i < m; ++i) H(i, k) = 0.0;
  }
  // implicit single-shift QR on the active window [lo, hi]
  const double eps = 2.220446049250313e-16;
  int hi = m - 1;
  int iter = 0;
  const int max_iter = 60 * m;
  while (hi > 0) {
    if (++iter > max_iter) return false;
    int lo = hi;
    while (lo > 0) {
      const double s = std::fabs(H(lo - 1, lo - 1)) + std::fabs(H(lo, lo));
      if (std::fabs(H(lo, lo - 1)) <= eps * (s > 0 ? s : 1.0)) {
        H(lo, lo - 1) = 0.0;
        break;
      }
      --lo;
    }
    if (lo == hi) {
      --hi;
      iter = 0;
      continue;
    }
    // Wilkinson shift from the trailing 2x2 block (real part if complex)
    const double a = H(hi - 1, hi - 1), b = H(hi - 1, hi), c = H(hi, hi - 1), d = H(hi, hi);
    const double tr = 0.5 * (a - d);
    const double disc = tr * tr + b * c;
    double mu;
    if (disc >= 0.0) {
      const double sq = std::sqrt(disc);
      mu = d - (b * c) / (tr + (tr >= 0 ? sq : -sq) + (tr == 0 && sq == 0 ? 1e-300 : 0.0));
    } else {
      mu = d + tr;  // real part of the complex pair
    }
    if (iter % 11 == 10) mu += std::fabs(H(hi, hi - 1));  // exceptional shift
    double x = H(lo, lo) - mu, z = H(lo + 1, lo);
    for (int k = lo; k < hi; ++k) {
      // (the entries of these operators stay far from overflow and underflow
      // when squared, so the plain root serves in place of hypot)
      const double r = std::sqrt(x * x + z * z);
      const double cs = r == 0.0 ? 1.0 : x / r, sn = r == 0.0 ? 0.0 : z / r;
      // rows k, k+1 (columns from max(lo, k-1) to m-1: full Schur form)
      for (int j = std::max(lo, k - 1); j < m; ++j) {
        const double h1 = H(k, j), h2 = H(k + 1, j);
        H(k, j) = cs * h1 + sn * h2;
        H(k + 1, j) = -sn * h1 + cs * h2;
      }
      // columns k, k+1 (rows 0 .. min(k+2, hi))
      const int rmax = std::min(k + 2, hi);
      for (int i = 0; i <= rmax; ++i) {
        const double h1 = H(i, k), h2 = H(i, k + 1);
        H(i, k) = cs * h1 + sn * h2;
        H(i, k + 1) = -sn * h1 + cs * h2;
      }
      double* z1r = Zr(k);
      double* z2r = Zr(k + 1);
      for (int i = 0; i < m; ++i) {
        const double z1 = z1r[i], z2 = z2r[i];
        z1r[i] = cs * z1 + sn * z2;
        z2r[i] = -sn * z1 + cs * z2;
      }
      if (k + 1 < hi) {
        x = H(k + 1, k);
        z = H(k + 2, k);
      }
    }
  }
  lam.assign(m, 0.0);
  for (int i = 0; i < m; ++i) lam[i] = H(i, i);
  // eigenvectors of the triangular T by back-substitution, then V = Z Y
  V.assign((size_t)m * m, 0.0);
  std::vector<double> y(m);
  double tnorm = 0.0;
  for (int i = 0; i < m; ++i)
    for (int j = i; j < m; ++j) tnorm = std::max(tnorm, std::fabs(H(i, j)));
  const double small = eps * (tnorm > 0 ? tnorm : 1.0);
  for (int k = 0; k < m; ++k) {
    for (int i = 0; i < m; ++i) y[i] = 0.0;
    y[k] = 1.0;
    for (int j = k - 1; j >= 0; --j) {
      double s = 0.0;
      for (int l = j + 1; l <= k; ++l) s += H(j, l) * y[l];
      double den = H(j, j) - lam[k];
      if (std::fabs(den) < small) den = den >= 0 ? small : -small;
      y[j] = -s / den;
    }
    // column k of V = Z y (l ascending for every i)
    std::fill(zs.begin(), zs.end(), 0.0);
    for (int l = 0; l <= k; ++l) {
      const double yl = y[l];
      const double* zr = Zr(l);
      for (int i = 0; i < m; ++i) zs[i] += zr[i] * yl;
    }
    double nrm = 0.0;
    for (int i = 0; i < m; ++i) nrm += zs[i] * zs[i];
    nrm = std::sqrt(nrm);
    for (int i = 0; i < m; ++i) V[(size_t)i * m + k] = zs[i] / nrm;
  }
  return true;
}

// Gauss-Jordan inverse with partial pivoting (m x m row-major)
bool invert(int m, const std::vector<double>& A, std::vector<double>& Ainv) {
  std::vector<double> W(A);
  Ainv.assign((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) Ainv[(size_t)i * m + i] = 1.0;
  for (int c = 0; c < m; ++c) {
    int piv = c;
    for (int r = c + 1; r < m; ++r)
      if (std::fabs(W[(size_t)r * m + c]) > std::fabs(W[(size_t)piv * m + c])) piv = r;
    if (W[(size_t)piv * m + c] == 0.0) return false;
    if (piv != c)
      for (int j = 0; j < m; ++j) {
        std::swap(W[(size_t)piv * m + j], W[(size_t)c * m + j]);
        std::swap(Ainv[(size_t)piv * m + j], Ainv[(size_t)c * m + j]);
      }
    // columns < c of W hold the identity by now, so W's rows change from column c on
    const double inv = 1.0 / W[(size_t)c * m + c];
    for (int j = c; j < m; ++j) W[(size_t)c * m + j] *= inv;
    for (int j = 0; j < m; ++j) Ainv[(size_t)c * m + j] *= inv;
    for (int r = 0; r < m; ++r) {
      if (r == c) continue;
      const double f = W[(size_t)r * m + c];
      if (f == 0.0) continue;
      double* wr = &W[(size_t)r * m];
      const double* wc = &W[(size_t)c * m];
      for (int j = c; j < m; ++j) wr[j] -= f * wc[j];
      double* ar = &Ainv[(size_t)r * m];
      const double* ac = &Ainv[(size_t)c * m];
      for (int j = 0; j < m; ++j) ar[j] -= f * ac[j];
    }
  }
  return true;
}

// Eigen-decomposition of a centro-symmetric A (J A J = A, J the exchange; the
// 1-D operator of an axis with the same face type at both ends).  With
// p = floor(m/2) and the orthogonal change of basis Q to symmetric vectors
// [u; sqrt(2) t; J u] / sqrt(2) and antisymmetric ones [u; 0; -J u] / sqrt(2),
// Q^T A Q = diag(S, W) with S = [A_aa + A_ab J, sqrt(2) a_ac; sqrt(2) a_ca, a_cc]
// (the centre row and column only for odd m) and W = A_aa - A_ab J, so the
// two half-size problems give V = Q diag(Vs, Vw) and V^{-1} = diag(Vs^{-1},
// Vw^{-1}) Q^T.  A's upper half is used (exact up to rounding for these).
bool eig_centro(int m, const std::vector<double>& A, std::vector<double>& lam, std::vector<double>& V,
                std::vector<double>& Vi) {
  const int p = m / 2, odd = m & 1, ps = p + odd;
  auto a = [&](int i, int j) { return A[(size_t)i * m + j]; };
  std::vector<double> S((size_t)ps * ps), W((size_t)p * p);
  const double r2 = std::sqrt(2.0);
  for (int i = 0; i < p; ++i)
    for (int j = 0; j < p; ++j) {
      const double ab = a(i, m - 1 - j);  // (A_ab J)_ij
      S[(size_t)i * ps + j] = a(i, j) + ab;
      W[(size_t)i * p + j] = a(i, j) - ab;
    }
  if (odd) {
    for (int i = 0; i < p; ++i) {
      S[(size_t)i * ps + p] = r2 * a(i, p);
      S[(size_t)p * ps + i] = r2 * a(p, i);
    }
    S[(size_t)p * ps + p] = a(p, p);
  }
  std::vector<double> ls, Vs, Vsi, lw, Vw, Vwi;
  // the two half-size problems are independent: the antisymmetric one on a
  // thread of its own
  bool okw = true;
  std::thread tw;
  if (p > 0) tw = std::thread([&]() { okw = eig_real(p, W, lw, Vw) && invert(p, Vw, Vwi); });
  const bool oks = eig_real(ps, S, ls, Vs) && invert(ps, Vs, Vsi);
  if (tw.joinable()) tw.join();
  if (!oks || !okw) return false;
  lam.assign(m, 0.0);
  V.assign((size_t)m * m, 0.0);
  Vi.assign((size_t)m * m, 0.0);
  const double h = 1.0 / r2;
  // symmetric eigenvectors: columns k < ps; antisymmetric: columns ps + k
  for (int k = 0; k < ps; ++k) {
    lam[k] = ls[k];
    for (int i = 0; i < p; ++i) {
      const double u = Vs[(size_t)i * ps + k] * h;
      V[(size_t)i * m + k] = u;
      V[(size_t)(m - 1 - i) * m + k] = u;
    }
    if (odd) V[(size_t)p * m + k] = Vs[(size_t)p * ps + k];
  }
  for (int k = 0; k < p; ++k) {
    lam[ps + k] = lw[k];
    for (int i = 0; i < p; ++i) {
      const double u = Vw[(size_t)i * p + k] * h;
      V[(size_t)i * m + ps + k] = u;
      V[(size_t)(m - 1 - i) * m + ps + k] = -u;
    }
  }
  // V^{-1} = diag(Vs^{-1}, Vw^{-1}) Q^T
  for (int k = 0; k < ps; ++k) {
    for (int j = 0; j < p; ++j) {
      const double u = Vsi[(size_t)k * ps + j] * h;
      Vi[(size_t)k * m + j] = u;
      Vi[(size_t)k * m + (m - 1 - j)] = u;
    }
    if (odd) Vi[(size_t)k * m + p] = Vsi[(size_t)k * ps + p];
  }
  for (int k = 0; k < p; ++k)
    for (int j = 0; j < p; ++j) {
      const double u = Vwi[(size_t)k * p + j] * h;
      Vi[(size_t)(ps + k) * m + j] = u;
      Vi[(size_t)(ps + k) * m + (m - 1 - j)] = -u;
    }
  return true;
}

// ---------------------------------------------------------------------------
// device kernels
// ---------------------------------------------------------------------------

// D(i, c) = sum_k A(i, k) B(k, c) per batch, arbitrary element strides; one
// wave computes a 16 x 64 tile with four 16x16 MFMA accumulators.
struct GemmArgs {
  const void* A;
  const void* B;
  void* D;
  int I, Kd, C;
  long long a_si, a_sk, b_sk, b_sc, d_si, d_sc;
  long long a_sb, b_sb, d_sb;  // batch strides
  int ps;                      // k_axis_gemm_split: the symmetric half, ceil(m / 2)
};

template <typename T>
__global__ __launch_bounds__(256) void k_axis_gemm(GemmArgs g) {
  typedef typename Mfma<T>::v4 v4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i0 = blockIdx.x * 16;
  const int c0 = (blockIdx.y * 4 + wave) * 64;
  const int b = blockIdx.z;
  const T* A = (const T*)g.A + b * g.a_sb;
  const T* B = (const T*)g.B + b * g.b_sb;
  T* D = (T*)g.D + b * g.d_sb;
  if (c0 >= g.C) return;
  const int li = lane & 15, lk = lane >> 4;  // A operand: row li, k lk; B operand: k lk, column li
  v4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = v4{0, 0, 0, 0};
  const int ia = i0 + li;
  for (int k0 = 0; k0 < g.Kd; k0 += 4) {
    const int k = k0 + lk;
    const T av = (ia < g.I && k < g.Kd) ? A[ia * g.a_si + k * g.a_sk] : T(0);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int c = c0 + t * 16 + li;
      const T bv = (c < g.C && k < g.Kd) ? B[k * g.b_sk + c * g.b_sc] : T(0);
      acc[t] = Mfma<T>::mac(av, bv, acc[t]);
    }
  }
  // lane holds column lane%16 of each 16x16 block; rows per Mfma<T>::row
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int c = c0 + t * 16 + li;
    if (c >= g.C) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + Mfma<T>::row(lk, r);
      if (i < g.I) D[i * g.d_si + c * g.d_sc] = acc[t][r];
    }
  }
}

// The same contraction for an axis whose 1-D operator is centro-symmetric
// (m = ps + ph, ps = ceil(m/2) a multiple of 16), with half the multiply-adds.
// With Q the symmetric / antisymmetric node-pair basis:
//   KIND 1 (the input enters through Q^T, e.g. V^{-1} = diag(Vs^{-1}, Vw^{-1}) Q^T):
//     output row i < ps (a symmetric mode) sums M[i][k] (x_k + x_{m-1-k}) over
//     k < ps, the middle node of odd m taken once; row i >= ps sums
//     M[i][k] (x_k - x_{m-1-k}) over k < ph;
//   KIND 2 (the output leaves through Q, e.g. V = Q diag(Vs, Vw)): for i < ps,
//     P = sum_{k < ps} M[i][k] y_k and R = sum_{k >= ps} M[i][k] y_k give node i
//     = P + R and node m-1-i = P - R (the middle node of odd m: P).
// M is read through the strides of either operand: ZSIDE, the contraction
// along the unit-stride axis, D[r][i] = sum_k X[r][k] M[i][k] (M the B
// operand, the split acts on the columns, each 16-column group symmetric or
// antisymmetric as a whole); otherwise D[i][c] = sum_k M[i][k] X[k][c] (M the
// A operand, each 16-row block one or the other).  One wave computes 16 rows x
// 64 columns of the output (KIND 2: of rows or columns below ps, with a second
// set of accumulators for R).
template <typename T, int KIND, bool ZSIDE>
__global__ __launch_bounds__(256) void k_axis_gemm_split(GemmArgs g) {
  typedef typename Mfma<T>::v4 v4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i0 = blockIdx.x * 16;
  const int c0 = (blockIdx.y * 4 + wave) * 64;
  const int b = blockIdx.z;
  const T* A = (const T*)g.A + b * g.a_sb;
  const T* B = (const T*)g.B + b * g.b_sb;
  T* D = (T*)g.D + b * g.d_sb;
  const int m = g.Kd, ps = g.ps, ph = m - g.ps;
  // output extent of this launch: rows (ZSIDE: columns) below ps for KIND 2
  const int I = (!ZSIDE && KIND == 2) ? ps : g.I;
  const int C = (ZSIDE && KIND == 2) ? ps : g.C;
  if (c0 >= C) return;
  const int li = lane & 15, lk = lane >> 4;
  const int ia = i0 + li;
  v4 acc[4], acr[KIND == 2 ? 4 : 1];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = v4{0, 0, 0, 0};
  if (KIND == 2)
#pragma unroll
    for (int t = 0; t < 4; ++t) acr[KIND == 2 ? t : 0] = v4{0, 0, 0, 0};
  if (KIND == 1) {
    // the row block (ZSIDE: each column group) is symmetric below ps
    const bool rsym = i0 < ps;
    const int kend = ZSIDE ? ps : (rsym ? ps : ph);
    for (int k0 = 0; k0 < kend; k0 += 4) {
      const int k = k0 + lk;
      const bool kin = k < kend;
      const int kr = m - 1 - (kin ? k : 0);  // mirror node (in range for k < ps)
      if (ZSIDE) {
        // A = X: pair sum and difference of this lane's row
        T sm = T(0), df = T(0);
        if (ia < I && kin) {
          const T x1 = A[ia * g.a_si + k * g.a_sk], x2 = A[ia * g.a_si + kr * g.a_sk];
          sm = kr == k ? x1 : x1 + x2;
          df = x1 - x2;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int cg = c0 + t * 16, c = cg + li;
          const bool csym = cg < ps;
          const bool kok = csym ? kin : k < ph;
          const T bv = (c < C && kok) ? B[k * g.b_sk + c * g.b_sc] : T(0);
          acc[t] = Mfma<T>::mac(csym ? sm : df, bv, acc[t]);
        }
      } else {
        const T av = (ia < I && kin) ? A[ia * g.a_si + k * g.a_sk] : T(0);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int c = c0 + t * 16 + li;
          T bv = T(0);
          if (c < C && kin) {
            const T x1 = B[k * g.b_sk + c * g.b_sc], x2 = B[kr * g.b_sk + c * g.b_sc];
            bv = rsym ? (kr == k ? x1 : x1 + x2) : x1 - x2;
          }
          acc[t] = Mfma<T>::mac(av, bv, acc[t]);
        }
      }
    }
  } else {
    // P over k < ps, R over k >= ps
    for (int k0 = 0; k0 < m; k0 += 4) {
      const int k = k0 + lk;
      const bool lower = k0 < ps;  // ps is a multiple of 16: no k-step straddles it
      const bool kin = k < m;
      const T av = (ia < I && kin) ? A[ia * g.a_si + k * g.a_sk] : T(0);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int c = c0 + t * 16 + li;
        const T bv = (c < C && kin) ? B[k * g.b_sk + c * g.b_sc] : T(0);
        if (lower) acc[t] = Mfma<T>::mac(av, bv, acc[t]);
        else acr[KIND == 2 ? t : 0] = Mfma<T>::mac(av, bv, acr[KIND == 2 ? t : 0]);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int c = c0 + t * 16 + li;
    if (c >= C) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + Mfma<T>::row(lk, r);
      if (i >= I) continue;
      if (KIND == 1) {
        D[i * g.d_si + c * g.d_sc] = acc[t][r];
      } else {
        const T P = acc[t][r], R = acr[KIND == 2 ? t : 0][r];
        if (ZSIDE) {
          D[i * g.d_si + c * g.d_sc] = P + R;
          if (c < ph) D[i * g.d_si + (m - 1 - c) * g.d_sc] = P - R;
        } else {
          D[i * g.d_si + c * g.d_sc] = P + R;
          if (i < ph) D[(m - 1 - i) * g.d_si + c * g.d_sc] = P - R;
        }
      }
    }
  }
}

// The same contractions (KIND 0 plain, 1 and 2 the even-odd split as above)
// with the operands staged through LDS: a workgroup of four waves computes a
// 64 x 64 output tile (each wave 32 x 32, 2 x 2 matrix-core blocks) over
// k-chunks of 16, so every loaded element feeds several matrix instructions.
// The split forms its pair sums and differences while staging; it needs ps a
// multiple of 64 so that a tile's rows (ZSIDE: columns) are all symmetric or
// all antisymmetric modes.
constexpr int kGt = 64, kGk = 16;  // output tile edge, k-chunk
template <typename T, int KIND, bool ZSIDE>
__global__ __launch_bounds__(256) void k_axis_gemm_lds(GemmArgs g) {
  typedef typename Mfma<T>::v4 v4;
  __shared__ T As[kGt][kGk + 1];
  __shared__ T Bs[kGk][kGt + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int i0 = blockIdx.x * kGt, c0 = blockIdx.y * kGt, b = blockIdx.z;
  const T* A = (const T*)g.A + b * g.a_sb;
  const T* B = (const T*)g.B + b * g.b_sb;
  T* D = (T*)g.D + b * g.d_sb;
  const int m = g.Kd, ps = g.ps, ph = m - g.ps;
  // output extent: rows (ZSIDE: columns) below ps for KIND 2
  const int I = (!ZSIDE && KIND == 2) ? ps : g.I;
  const int C = (ZSIDE && KIND == 2) ? ps : g.C;
  // KIND 1: the tile's modes are symmetric below ps; their k range
  const bool tsym = ZSIDE ? c0 < ps : i0 < ps;
  const int kend = KIND == 1 ? (tsym ? ps : ph) : m;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  v4 acc[2][2], acr[KIND == 2 ? 2 : 1][KIND == 2 ? 2 : 1];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      acc[x][y] = v4{0, 0, 0, 0};
      if (KIND == 2) acr[KIND == 2 ? x : 0][KIND == 2 ? y : 0] = v4{0, 0, 0, 0};
    }
  for (int k0 = 0; k0 < kend; k0 += kGk) {
    // stage A (64 rows x 16 k) and B (16 k x 64 columns), zero outside
#pragma unroll
    for (int q = 0; q < kGt * kGk / 256; ++q) {
      const int e = tid + q * 256;
      const int r = e / kGk, kk = e - r * kGk;
      const int i = i0 + r, k = k0 + kk;
      T v = T(0);
      if (i < I && k < kend) {
        v = A[i * g.a_si + k * g.a_sk];
        if (KIND == 1 && ZSIDE) {
          const int kr = m - 1 - k;
          const T x2 = A[i * g.a_si + kr * g.a_sk];
          v = tsym ? (kr == k ? v : v + x2) : v - x2;
        }
      }
      As[r][kk] = v;
    }
#pragma unroll
    for (int q = 0; q < kGt * kGk / 256; ++q) {
      const int e = tid + q * 256;
      const int kk = e / kGt, cc = e - kk * kGt;
      const int k = k0 + kk, c = c0 + cc;
      T v = T(0);
      if (c < C && k < kend) {
        v = B[k * g.b_sk + c * g.b_sc];
        if (KIND == 1 && !ZSIDE) {
          const int kr = m - 1 - k;
          const T x2 = B[kr * g.b_sk + c * g.b_sc];
          v = tsym ? (kr == k ? v : v + x2) : v - x2;
        }
      }
      Bs[kk][cc] = v;
    }
    __syncthreads();
    const bool upper = KIND == 2 && k0 >= ps;  // ps is a multiple of 16: chunks do not straddle it
#pragma unroll
    for (int ks = 0; ks < kGk / 4; ++ks) {
      T av[2], bv[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) av[x] = As[wr + x * 16 + li][ks * 4 + lk];
#pragma unroll
      for (int y = 0; y < 2; ++y) bv[y] = Bs[ks * 4 + lk][wc + y * 16 + li];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          if (upper) acr[KIND == 2 ? x : 0][KIND == 2 ? y : 0] =
              Mfma<T>::mac(av[x], bv[y], acr[KIND == 2 ? x : 0][KIND == 2 ? y : 0]);
          else acc[x][y] = Mfma<T>::mac(av[x], bv[y], acc[x][y]);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      const int c = c0 + wc + y * 16 + li;
      if (c >= C) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wr + x * 16 + Mfma<T>::row(lk, r);
        if (i >= I) continue;
        if (KIND != 2) {
          D[i * g.d_si + c * g.d_sc] = acc[x][y][r];
        } else {
          const T P = acc[x][y][r], R = acr[KIND == 2 ? x : 0][KIND == 2 ? y : 0][r];
          D[i * g.d_si + c * g.d_sc] = P + R;
          if (ZSIDE ? c < ph : i < ph) {
            if (ZSIDE) D[i * g.d_si + (m - 1 - c) * g.d_sc] = P - R;
            else D[(m - 1 - i) * g.d_si + c * g.d_sc] = P - R;
          }
        }
      }
    }
}

// Contraction of packed blocks along one axis with a dense m x m matrix,
// y_i = sum_k M[i][k] x_k per pencil (M^T with trans), for m <= MP <= 128, on
// the matrix cores (MFMA 16x16x4).  One wave owns a task of 16 pencils and
// computes every output row of them: the pencils' values are the B operand,
// loaded once from memory straight into registers in MFMA layout; the A
// operand -- M cut into 16-row blocks and 4-wide k-steps, zero past m -- comes
// from a fragment table that the workgroup copies into LDS once (written on
// the host at setup, one table per axis, side and transposition).  Nothing is
// exchanged between waves, so a workgroup synchronises only after the table
// copy; each wave streams its tasks (loads, 8 x KS matrix-core steps, stores).
//
// The k order of the steps is the row order of the accumulator layout of the
// same type (fdm_kmap), so that the output of one contraction, held in
// registers, is the B operand of another: the middle pair -- the last forward
// and the first backward contraction, both along the same axis, with the
// eigenvalue scaling between them -- runs as one kernel.
//
// Input and output are each either packed interior blocks (nb blocks of
// m0 x m1 x m2 back to back) or full fields (n_a = m_a + 2 nodes per axis, the
// interior block at node offset (1,1,1), field b at offs[b]), so the packing
// of the first contraction and the unpacking of the last one are part of
// them; the last one (full output) also zeroes the boundary nodes of its
// fields.  With lam set, the output is divided by Kc (lam0[i0] + lam1[i1] +
// lam2[i2]): the eigenvalue scaling between the two halves of the
// preconditioner.
struct FdmArgs {
  const int* gate;            // null, or a device flag: the contraction does nothing while it reads 0
  const void* tab;            // fragment table of the (first) contraction
  const void* tab2;           // fragment table of the middle pair's second contraction
  const void* X;
  void* Y;
  int m, axis, nb;
  int m0, m1, m2;             // dims of one packed block
  const long long* offs;      // full layouts: field b starts at offs[b] (null: b * n0 n1 n2)
  const void* lam0;           // eigenvalues per axis (scaling)
  const void* lam1;
  const void* lam2;
  double inv_k;               // 1 / Kc of a single system (sys == null)
  const int* sys;             // batch: Kc of block b is kc[sys[b]]
  const double* kc;
};

// fusion modes: X is a full field / Y is a full field / Y is scaled / the
// middle pair (first table, scaling, second table)
enum { FDM_XFULL = 1, FDM_YFULL = 2, FDM_SCALE = 4, FDM_MID = 8 };

// KIND of one contraction (axes whose 1-D operator is centro-symmetric, so
// that the factors are V = Q diag(Vs, Vw) and V^{-1} = diag(Vs^{-1}, Vw^{-1}) Q^T
// with Q the symmetric / antisymmetric node-pair basis; modes ordered
// symmetric first):
//   0  plain: every row block runs the whole k range;
//   1  the input enters through Q^T: the operand is the pair sums
//      x_j + x_{m-1-j} (the middle node of odd m kept) for the symmetric row
//      blocks and the differences for the antisymmetric ones;
//   2  the output leaves through Q: row i of the symmetric blocks is a_i, of
//      the antisymmetric ones b_i (same lane and register), and node i
//      receives a_i + b_i, node m-1-i a_i - b_i, the middle node a_p.
// Kinds 1 and 2 do half the multiply-adds; they need ps = ceil(m/2) to be a
// multiple of 16, and then ps = MP/2.  The middle pair takes SPLIT 3: kind 1
// for the first table, kind 2 for the second (SPLIT 0: both plain).

// k-index of MFMA step ks for lane group lk (lane / 16): the row that the
// accumulator of the same type holds in register ks % 4 of row block ks / 4
__host__ __device__ constexpr int fdm_kmap(int ks, int lk, bool f32) {
  return f32 ? 16 * (ks / 4) + 4 * lk + (ks % 4) : 4 * ks + lk;
}

// linear offset of boundary node u of an n0 x n1 x n2 field (faces x, y, z)
__device__ inline long long face_node(long long u, int n0, int n1, int n2) {
  const long long fxy = (long long)n1 * n2, fxz = (long long)n0 * n2, fyz = (long long)n0 * n1;
  int i, j, k;
  if (u < 2 * fxy) {  // x faces
    i = u < fxy ? 0 : n0 - 1;
    u %= fxy;
    j = (int)(u / n2);
    k = (int)(u % n2);
  } else if ((u -= 2 * fxy) < 2 * fxz) {  // y faces
    j = u < fxz ? 0 : n1 - 1;
    u %= fxz;
    i = (int)(u / n2);
    k = (int)(u % n2);
  } else {  // z faces
    u -= 2 * fxz;
    k = u < fyz ? 0 : n2 - 1;
    u %= fyz;
    i = (int)(u / n1);
    j = (int)(u % n1);
  }
  return ((long long)i * n1 + j) * n2 + k;
}

// fragment-table sizes (elements) of one contraction of padded width MP
__host__ __device__ constexpr int fdm_tab_elems(int MP, int kind) { return (MP / 16) * (kind ? MP / 8 : MP / 4) * 64; }

constexpr int kFdmWaves = 4;  // waves per workgroup

template <typename T>
__host__ __device__ constexpr int fdm_lds_bytes(int MP, int MODE, int SPLIT) {
  const bool mid = MODE & FDM_MID;
  const int ka = mid ? (SPLIT ? 1 : 0) : SPLIT, kb = mid ? (SPLIT ? 2 : 0) : 0;
  return (fdm_tab_elems(MP, ka) + (mid ? fdm_tab_elems(MP, kb) : 0) + ((MODE & FDM_SCALE) ? 3 * 128 : 0)) *
         (int)sizeof(T);
}

// N 16-byte words from global memory into LDS by the workgroup, in rounds of
// at most 16 loads per lane that are all issued before the first store
template <int N>
__device__ __forceinline__ void copy_to_lds(const int4* __restrict__ src, int4* dst, int tid) {
  static_assert(N > 0, "empty table");
  constexpr int NT = 64 * kFdmWaves, PER = (N + NT - 1) / NT, R = PER < 16 ? PER : 16;
#pragma unroll
  for (int base = 0; base < PER; base += R) {
    int4 v[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int e = tid + (base + i) * NT;
      v[i] = src[e < N ? e : N - 1];  // unconditional: the loads stay in registers
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int e = tid + (base + i) * NT;
      if (e < N) dst[e] = v[i];
    }
  }
}

// the eigenvalue scaling v / (Kc (lam_transverse + lam_i)), ik = 1 / Kc: FP64
// divides exactly; FP32 multiplies by the hardware reciprocal (1 ulp), which the
// FP32 preconditioner's accuracy does not notice
template <typename T>
__device__ __forceinline__ T fdm_scale(T v, double ik, double sc, T lam) {
  if constexpr (sizeof(T) == sizeof(float)) {
    return v * float(ik) * __builtin_amdgcn_rcpf(float(sc) + lam);
  } else {
    return T(double(v) * ik / (sc + double(lam)));
  }
}

// acc[rb] (16 rows of row block rb, every rb) = table x B, k-step by k-step
// (KIND 0: KF steps; kinds 1, 2: KH steps, the symmetric blocks taking one
// operand, the antisymmetric ones the other).  MASKED: B holds the pencil's
// raw loads (see k_fdm_wave's load()), turned into operands here, one step at
// a time, so that each step waits only for its own loads; otherwise B holds
// the operands themselves (B[ks] and, kinds 1 and 2, B[KH + ks]).
template <typename T, int KIND, int NB, int KF, int KH, bool MASKED>
__device__ __forceinline__ void contract(const T* __restrict__ tab, int lane, const T (&B)[KF],
                                         typename Mfma<T>::v4 (&acc)[NB], int lk, int m, bool valid) {
  constexpr int NKS = KIND ? KH : KF;
  constexpr bool F32 = sizeof(T) == sizeof(float);
  const int ps = (m + 1) / 2, ph = m / 2;
#pragma unroll
  for (int rb = 0; rb < NB; ++rb) acc[rb] = typename Mfma<T>::v4{0, 0, 0, 0};
#pragma unroll
  for (int ks = 0; ks < NKS; ++ks) {
    // one step's table reads at a time: hoisting more only costs registers
    __builtin_amdgcn_sched_barrier(0);
    const int j = fdm_kmap(ks, lk, F32);
    T bs, ba;  // operand of the symmetric (or every) row block, of the antisymmetric ones
    if constexpr (!MASKED) {
      bs = B[ks];
      ba = KIND ? B[KH + ks] : bs;
    } else if constexpr (KIND == 1) {
      // pair sums and differences; the middle node of odd m (j = ph) stands alone
      const T xj = B[ks], xr = B[KH + ks];
      bs = valid ? (j < ph ? xj + xr : xj) : T(0);
      ba = valid && j < ph ? xj - xr : T(0);
    } else if constexpr (KIND == 2) {
      bs = valid ? B[ks] : T(0);
      ba = valid && ps + j < m ? B[KH + ks] : T(0);
    } else {
      bs = valid && j < m ? B[ks] : T(0);
      ba = bs;
    }
#pragma unroll
    for (int rb = 0; rb < NB; ++rb)
      acc[rb] = Mfma<T>::mac(tab[(rb * NKS + ks) * 64 + lane], (KIND && rb >= NB / 2) ? ba : bs, acc[rb]);
  }
}

template <typename T, int MP, int MODE, int SPLIT>
__global__ __launch_bounds__(64 * kFdmWaves) void k_fdm_wave(FdmArgs g) {
  if (g.gate && !*g.gate) return;
  constexpr int NB = MP / 16, KF = MP / 4, KH = MP / 8;
  constexpr bool F32 = sizeof(T) == sizeof(float);
  constexpr bool XF = MODE & FDM_XFULL, YF = MODE & FDM_YFULL, SCL = MODE & FDM_SCALE, MID = MODE & FDM_MID;
  constexpr bool FULL = XF || YF;
  constexpr int SA = MID ? (SPLIT ? 1 : 0) : SPLIT;  // kind of the first (or only) contraction
  constexpr int SB = MID ? (SPLIT ? 2 : 0) : 0;      // kind of the second one
  constexpr int TA = fdm_tab_elems(MP, SA), TB = MID ? fdm_tab_elems(MP, SB) : 0;
  static_assert(!MID || SCL, "the middle pair scales between its contractions");
  static_assert(!MID || SPLIT == 0 || SPLIT == 3, "middle pair: SPLIT 0 or 3");
  static_assert(MID || SPLIT <= 2, "SPLIT 3 is the middle pair's");
  static_assert(SPLIT == 0 || MP >= 32, "split contractions need two row blocks");
  typedef typename Mfma<T>::v4 V4;
  extern __shared__ __align__(16) unsigned char smem[];
  T* tabA = (T*)smem;
  T* tabB = tabA + TA;
  T* lam_s = tabB + TB;  // SCL: every axis' eigenvalues, 128 each
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int m = g.m, axis = g.axis;
  const T* X = (const T*)g.X;
  T* Y = (T*)g.Y;
  const int n0 = g.m0 + 2, n1 = g.m1 + 2, n2 = g.m2 + 2;
  const int plane = g.m1 * g.m2, bsz = plane * g.m0;
  const int fplane = n1 * n2, fsz = fplane * n0;
  const int pstride = axis == 2 ? 1 : axis == 1 ? g.m2 : plane;  // packed
  const int fstride = axis == 2 ? 1 : axis == 1 ? n2 : fplane;   // full
  const int sxa = XF ? fstride : pstride, sya = YF ? fstride : pstride;
  const int ppb = bsz / m;  // pencils per block
  const int npen = ppb * g.nb;
  const int ntasks = (npen + 15) / 16;
  const int ps = (m + 1) / 2, ph = m / 2;  // symmetric / antisymmetric halves (split kinds: ps = MP/2)

  // this lane's pencil of a task: its first element in X and Y, and (scaling)
  // the block's 1 / Kc and the pencil's indices across the axis
  bool valid = false;
  long long bx = 0, by = 0;
  int ia = 0, ib = 0, bi = 0;
  auto locate = [&](int task) {
    const int q = task * 16 + li;
    valid = q < npen;
    if (!valid) return;
    bi = q / ppb;
    const int qq = q - bi * ppb;
    int i0 = 0, i1 = 0, i2 = 0;  // interior indices (axis index 0)
    if (axis == 0) {
      i1 = qq / g.m2;
      i2 = qq - i1 * g.m2;
    } else if (axis == 1) {
      i0 = qq / g.m2;
      i2 = qq - i0 * g.m2;
    } else {
      i0 = qq / g.m1;
      i1 = qq - i0 * g.m1;
    }
    const long long pk = (long long)bi * bsz + ((long long)i0 * g.m1 + i1) * g.m2 + i2;
    long long fk = 0;
    if (FULL) fk = (g.offs ? g.offs[bi] : (long long)bi * fsz) + ((long long)(i0 + 1) * n1 + (i1 + 1)) * n2 + (i2 + 1);
    bx = XF ? fk : pk;
    by = YF ? fk : pk;
    ia = axis == 0 ? i1 : i0;  // the first transverse axis' index
    ib = axis == 2 ? i1 : i2;  // the second one's
  };
  // the B operand's raw loads: row fdm_kmap(ks, lk) of the pencil at step ks
  // (kind 1: and its mirror node m-1-j for the pair sums and differences;
  // kind 2: the first ps rows, then the rest).  Every load is issued, rows past
  // the pencil clamped to its last node and invalid lanes reading element 0, so
  // the number in flight is static and the matrix-core steps wait only for
  // their own loads; contract() masks the values it does not use.
  T B[KF];
  auto load = [&]() {
    if (SA == 1) {
#pragma unroll
      for (int ks = 0; ks < KH; ++ks) {
        const int j = fdm_kmap(ks, lk, F32);  // < ps
        const int jr = j < ph ? m - 1 - j : j;
        B[ks] = X[bx + (long long)j * sxa];
        B[KH + ks] = X[bx + (long long)jr * sxa];
      }
    } else if (SA == 2) {
#pragma unroll
      for (int ks = 0; ks < KH; ++ks) {
        const int j = fdm_kmap(ks, lk, F32);
        const int j2 = ps + j < m ? ps + j : m - 1;
        B[ks] = X[bx + (long long)j * sxa];
        B[KH + ks] = X[bx + (long long)j2 * sxa];
      }
    } else {
#pragma unroll
      for (int ks = 0; ks < KF; ++ks) {
        const int j = fdm_kmap(ks, lk, F32);
        B[ks] = X[bx + (long long)(j < m ? j : m - 1) * sxa];
      }
    }
  };  // the fragment tables (and eigenvalues) into LDS, 16 bytes per lane, the
  // loads of a table in flight together (a load-store loop would pay the L2
  // latency once per iteration); before the first task's operand loads, which
  // would hold the table's loads back behind memory latency
  copy_to_lds<TA * (int)sizeof(T) / 16>((const int4*)g.tab, (int4*)tabA, tid);
  if constexpr (MID) copy_to_lds<TB * (int)sizeof(T) / 16>((const int4*)g.tab2, (int4*)tabB, tid);
  if constexpr (SCL) {
    const T* lp[3] = {(const T*)g.lam0, (const T*)g.lam1, (const T*)g.lam2};
    const int md[3] = {g.m0, g.m1, g.m2};
    for (int e = tid; e < 3 * 128; e += 64 * kFdmWaves) {
      const int a = e / 128, i = e - a * 128;
      lam_s[e] = i < md[a] ? lp[a][i] : T(0);
    }
  }
  // the first task's operand, in flight across the barrier
  int task = blockIdx.x * kFdmWaves + wave;
  if (task < ntasks) {
    locate(task);
    load();
  }
  if (YF) {
    // the boundary nodes of the output fields (the contraction writes the interior)
    const long long faces = 2LL * ((long long)n1 * n2 + (long long)n0 * n2 + (long long)n0 * n1);
    for (long long t = (long long)blockIdx.x * 64 * kFdmWaves + tid; t < faces * g.nb;
         t += (long long)gridDim.x * 64 * kFdmWaves) {
      const int b = (int)(t / faces);
      const long long fo = g.offs ? g.offs[b] : (long long)b * fsz;
      Y[fo + face_node(t - b * faces, n0, n1, n2)] = T(0);
    }
  }
  // a barrier over the LDS stores only: a full __syncthreads() would also wait
  // for the operand loads just issued, which are meant to land during the
  // first matrix-core steps
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  for (; task < ntasks; task += gridDim.x * kFdmWaves) {
    // every row block at once, k-step by k-step: eight independent
    // accumulation chains, started as soon as the first rows arrive
    V4 acc[NB];
    contract<T, SA, NB, KF, KH, true>(tabA, lane, B, acc, lk, m, valid);
    if constexpr (MID) {
      // the first contraction, scaled, is the second one's B operand
      const int a0 = axis == 0 ? 1 : 0, a1 = axis == 2 ? 1 : 2;
      const double sc = valid ? double(lam_s[a0 * 128 + ia]) + double(lam_s[a1 * 128 + ib]) : 0.0;
      const double ik = valid ? (g.sys ? 1.0 / g.kc[g.sys[bi]] : g.inv_k) : 0.0;
#pragma unroll
      for (int rb = 0; rb < NB; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * rb + Mfma<T>::row(lk, r);
          B[4 * rb + r] = i < m ? fdm_scale<T>(acc[rb][r], ik, sc, lam_s[axis * 128 + i]) : T(0);
        }
      contract<T, SB, NB, KF, KH, false>(tabB, lane, B, acc, lk, m, valid);
    } else if constexpr (SCL) {
      const int a0 = axis == 0 ? 1 : 0, a1 = axis == 2 ? 1 : 2;
      const double sc = valid ? double(lam_s[a0 * 128 + ia]) + double(lam_s[a1 * 128 + ib]) : 0.0;
      const double ik = valid ? (g.sys ? 1.0 / g.kc[g.sys[bi]] : g.inv_k) : 0.0;
#pragma unroll
      for (int rb = 0; rb < NB; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * rb + Mfma<T>::row(lk, r);
          if (i < m) acc[rb][r] = fdm_scale<T>(acc[rb][r], ik, sc, lam_s[axis * 128 + i]);
        }
    }
    constexpr int SOUT = MID ? SB : SA;  // the kind whose outputs are stored
    if (valid) {
      if constexpr (SOUT == 2) {
        // rows i of the symmetric blocks hold a_i, of the antisymmetric ones b_i
#pragma unroll
        for (int rb = 0; rb < NB / 2; ++rb)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = 16 * rb + Mfma<T>::row(lk, r);
            const T a = acc[rb][r], b = acc[rb + NB / 2][r];
            if (i < ph) {
              Y[by + (long long)i * sya] = a + b;
              Y[by + (long long)(m - 1 - i) * sya] = a - b;
            } else if (i < ps) {
              Y[by + (long long)i * sya] = a;  // the middle node of odd m
            }
          }
      } else {
#pragma unroll
        for (int rb = 0; rb < NB; ++rb)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = 16 * rb + Mfma<T>::row(lk, r);
            if (i < m) Y[by + (long long)i * sya] = acc[rb][r];
          }
      }
    }
    if (task + gridDim.x * kFdmWaves < ntasks) {
      locate(task + gridDim.x * kFdmWaves);
      load();
    }
  }
}

template <typename T>
__global__ void k_pack_interior(const T* __restrict__ in, T* __restrict__ out, int n0, int n1, int n2) {
  const int m0 = n0 - 2, m1 = n1 - 2, m2 = n2 - 2;
  const size_t tot = (size_t)m0 * m1 * m2;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(t % m2);
    const size_t r = t / m2;
    const int j = (int)(r % m1), i = (int)(r / m1);
    out[t] = in[((size_t)(i + 1) * n1 + (j + 1)) * n2 + (k + 1)];
  }
}

template <typename T>
__global__ void k_unpack_interior(const T* __restrict__ in, T* __restrict__ out, int n0, int n1, int n2) {
  const size_t tot = (size_t)n0 * n1 * n2;
  const int m1 = n1 - 2, m2 = n2 - 2;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(t % n2);
    const size_t r = t / n2;
    const int j = (int)(r % n1), i = (int)(r / n1);
    T v = T(0);
    if (i > 0 && i < n0 - 1 && j > 0 && j < n1 - 1 && k > 0 && k < n2 - 1)
      v = in[((size_t)(i - 1) * m1 + (j - 1)) * m2 + (k - 1)];
    out[t] = v;
  }
}

template <typename T>
__global__ void k_eig_scale(T* x, const T* lx, const T* ly, const T* lz, double inv_k, int m0, int m1, int m2) {
  const size_t tot = (size_t)m0 * m1 * m2;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(t % m2);
    const size_t r = t / m2;
    const int j = (int)(r % m1), i = (int)(r / m1);
    x[t] = T(double(x[t]) * inv_k / (double(lx[i]) + double(ly[j]) + double(lz[k])));
  }
}

// batched variants: member k of a group reads / writes the packed field at
// offs[k] and owns block k of the packed interior buffers
template <typename T>
__global__ void k_pack_interior_b(const T* __restrict__ in, const long long* __restrict__ offs, T* __restrict__ out,
                                  int n0, int n1, int n2) {
  const int m0 = n0 - 2, m1 = n1 - 2, m2 = n2 - 2;
  const size_t tot = (size_t)m0 * m1 * m2;
  const T* src = in + offs[blockIdx.y];
  T* dst = out + (size_t)blockIdx.y * tot;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(t % m2);
    const size_t r = t / m2;
    const int j = (int)(r % m1), i = (int)(r / m1);
    dst[t] = src[((size_t)(i + 1) * n1 + (j + 1)) * n2 + (k + 1)];
  }
}

template <typename T>
__global__ void k_unpack_interior_b(const T* __restrict__ in, const long long* __restrict__ offs, T* __restrict__ out,
                                    int n0, int n1, int n2) {
  const size_t tot = (size_t)n0 * n1 * n2;
  const int m1 = n1 - 2, m2 = n2 - 2;
  const T* src = in + (size_t)blockIdx.y * (size_t)(n0 - 2) * m1 * m2;
  T* dst = out + offs[blockIdx.y];
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(t % n2);
    const size_t r = t / n2;
    const int j = (int)(r % n1), i = (int)(r / n1);
    T v = T(0);
    if (i > 0 && i < n0 - 1 && j > 0 && j < n1 - 1 && k > 0 && k < n2 - 1)
      v = src[((size_t)(i - 1) * m1 + (j - 1)) * m2 + (k - 1)];
    dst[t] = v;
  }
}

template <typename T>
__global__ void k_eig_scale_b(T* x, const T* lx, const T* ly, const T* lz, const int* __restrict__ sys,
                              const double* __restrict__ kc, int m0, int m1, int m2) {
  const size_t tot = (size_t)m0 * m1 * m2;
  T* xb = x + (size_t)blockIdx.y * tot;
  const double inv_k = 1.0 / kc[sys[blockIdx.y]];
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(t % m2);
    const size_t r = t / m2;
    const int j = (int)(r % m1), i = (int)(r / m1);
    xb[t] = T(double(xb[t]) * inv_k / (double(lx[i]) + double(ly[j]) + double(lz[k])));
  }
}

inline int grid1(size_t n) {
  size_t g = (n + 1023) / 1024;
  return (int)std::max<size_t>(1, std::min<size_t>(g, 8192));
}

}  // namespace

// ---------------------------------------------------------------------------
// plan-level setup and application
// ---------------------------------------------------------------------------

// Fragment table of one contraction (see k_fdm_wave): entry (rb * KS + ks) * 64
// + lane is the A operand of row block rb at step ks for that lane: M (M^T with
// tr) at row 16 rb + lane % 16 and column fdm_kmap(ks, lane / 16), with the
// half-matrix indexing of the even-odd kinds, zero outside.  M is m x m,
// row-major.
static void fdm_table(const double* M, int m, int mp, int kind, bool tr, bool f32, double* out) {
  const int nbk = mp / 16, nks = kind ? mp / 8 : mp / 4;
  const int ps = (m + 1) / 2, ph = m / 2;
  for (int rb = 0; rb < nbk; ++rb)
    for (int ks = 0; ks < nks; ++ks)
      for (int lane = 0; lane < 64; ++lane) {
        const int row = 16 * rb + (lane & 15), k = fdm_kmap(ks, lane >> 4, f32);
        const bool anti = kind != 0 && 16 * rb >= ps;
        int r = row, col = k;
        bool ok = row < m && k < m;
        if (kind == 1) {
          ok = row < m && k < (anti ? ph : ps);
        } else if (kind == 2) {
          r = anti ? row - ps : row;
          col = anti ? ps + k : k;
          ok = r < (anti ? ph : ps) && k < (anti ? ph : ps);
        }
        out[((size_t)rb * nks + ks) * 64 + lane] = ok ? (tr ? M[(size_t)col * m + r] : M[(size_t)r * m + col]) : 0.0;
      }
}

int precond_setup(cheb_plan* p) {
  if (p->pc_ready) return CHEB_OK;
  size_t off64 = 0;
  std::vector<double> host;
  PrecondAxis ax[3] = {};
  // axes with the same 1-D problem (N, L, face pair) share one decomposition;
  // the distinct ones are decomposed on host threads of their own
  int src[3];
  for (int a = 0; a < 3; ++a) {
    src[a] = a;
    for (int b = 0; b < a; ++b)
      if (src[b] == b && p->ax[b].N == p->ax[a].N && p->ax[b].L == p->ax[a].L &&
          p->g.bc[2 * b] == p->g.bc[2 * a] && p->g.bc[2 * b + 1] == p->g.bc[2 * a + 1] &&
          face_sigma(p, 2 * b) == face_sigma(p, 2 * a) && face_sigma(p, 2 * b + 1) == face_sigma(p, 2 * a + 1)) {
        src[a] = b;
        break;
      }
  }
  std::vector<double> lamv[3], Vv[3], Viv[3];
  bool okv[3] = {true, true, true};
  {
    std::vector<std::thread> th;
    for (int a = 0; a < 3; ++a) {
      if (src[a] != a) continue;
      th.emplace_back([&, a]() {
        const int m = p->ax[a].N - 1;
        std::vector<double> A;
        reduced_1d(p->ax[a].N, p->ax[a].L, p->g.bc[2 * a], p->g.bc[2 * a + 1], face_sigma(p, 2 * a),
                   face_sigma(p, 2 * a + 1), A);
        // the same face row at both ends: the 1-D operator is centro-symmetric
        const bool centro = p->g.bc[2 * a] == p->g.bc[2 * a + 1] && face_sigma(p, 2 * a) == face_sigma(p, 2 * a + 1);
        okv[a] = centro ? eig_centro(m, A, lamv[a], Vv[a], Viv[a])
                                                      : eig_real(m, A, lamv[a], Vv[a]) && invert(m, Vv[a], Viv[a]);
      });
    }
    for (auto& t : th) t.join();
  }
  for (int a = 0; a < 3; ++a) {
    const int N = p->ax[a].N, m = N - 1;
    if (!okv[src[a]]) {
      set_error("preconditioner setup: eigen-decomposition failed");
      return CHEB_ERR_UNSUPPORTED;
    }
    const std::vector<double>& lam = lamv[src[a]];
    const std::vector<double>& V = Vv[src[a]];
    const std::vector<double>& Vi = Viv[src[a]];
    ax[a].m = m;
    // the even-odd contraction needs the centro-symmetric factors and whole
    // 16-row halves
    const int sa = src[a];
    const bool centro_a = p->g.bc[2 * sa] == p->g.bc[2 * sa + 1] && face_sigma(p, 2 * sa) == face_sigma(p, 2 * sa + 1);
    ax[a].split = centro_a && m <= 128 && ((m + 1) / 2) % 16 == 0 ? 1 : 0;
    ax[a].centro = centro_a ? 1 : 0;
    ax[a].off_V = off64;
    host.insert(host.end(), V.begin(), V.end());
    off64 += (size_t)m * m;
    ax[a].off_Vi = off64;
    host.insert(host.end(), Vi.begin(), Vi.end());
    off64 += (size_t)m * m;
    ax[a].off_lam = off64;
    host.insert(host.end(), lam.begin(), lam.end());
    off64 += (size_t)m;
  }
  // fragment tables of the matrix-core contractions: each side (V^{-1}, V)
  // plain and transposed, in the k order of each precision's accumulator
  // layout (so the FP32 tables are written separately)
  struct TabJob {
    int a, dir, tr, kind;
    size_t off;
  };
  std::vector<TabJob> jobs;
  for (int a = 0; a < 3; ++a) {
    const int m = ax[a].m;
    if (m > 128) continue;
    if (src[a] != a) {
      // the same 1-D problem as an earlier axis: the same tables
      for (int dir = 0; dir < 2; ++dir)
        for (int tr = 0; tr < 2; ++tr) ax[a].off_tab[dir][tr] = ax[src[a]].off_tab[dir][tr];
      continue;
    }
    const int mp = 16 * ((m + 15) / 16);
    for (int dir = 0; dir < 2; ++dir)
      for (int tr = 0; tr < 2; ++tr) {
        off64 = (off64 + 3) / 4 * 4;  // 16-byte aligned in both precisions
        const int kind = ax[a].split ? dir + 1 : 0;
        ax[a].off_tab[dir][tr] = off64;
        jobs.push_back({a, dir, tr, kind, off64});
        off64 += fdm_tab_elems(mp, kind);
      }
  }
  host.resize(off64, 0.0);
  std::vector<float> host32(host.size());
  for (size_t i = 0; i < host.size(); ++i) host32[i] = float(host[i]);
  for (const TabJob& j : jobs) {
    const int m = ax[j.a].m, mp = 16 * ((m + 15) / 16);
    // the V^{-1} side applies V^{-1} (V^T when transposed), the V side V (V^{-1} T)
    const double* M = host.data() + ((j.dir == 0) != (j.tr != 0) ? ax[j.a].off_Vi : ax[j.a].off_V);
    std::vector<double> t(fdm_tab_elems(mp, j.kind));
    fdm_table(M, m, mp, j.kind, j.tr != 0, false, t.data());
    std::copy(t.begin(), t.end(), host.begin() + j.off);
    fdm_table(M, m, mp, j.kind, j.tr != 0, true, t.data());
    for (size_t i = 0; i < t.size(); ++i) host32[j.off + i] = float(t[i]);
  }
  int rc = hip_check(hipMalloc((void**)&p->pc64, host.size() * sizeof(double)), "hipMalloc(preconditioner)");
  if (!rc) rc = hip_check(hipMalloc((void**)&p->pc32, host.size() * sizeof(float)), "hipMalloc(preconditioner)");
  if (!rc)
    rc = hip_check(hipMemcpy(p->pc64, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice),
                   "hipMemcpy(preconditioner)");
  if (!rc)
    rc = hip_check(hipMemcpy(p->pc32, host32.data(), host32.size() * sizeof(float), hipMemcpyHostToDevice),
                   "hipMemcpy(preconditioner)");
  if (rc) return rc;
  for (int a = 0; a < 3; ++a) p->pc_ax[a] = ax[a];
  p->pc_ready = 1;
  return CHEB_OK;
}

template <typename T>
static const T* pc_base(const cheb_plan* p);
template <>
const double* pc_base<double>(const cheb_plan* p) { return p->pc64; }
template <>
const float* pc_base<float>(const cheb_plan* p) { return p->pc32; }

// persistent launch: at most as many workgroups as the device holds at once
// (queried once per instantiation and device), no more than the tasks need
template <typename T, int MP, int MODE, int SPLIT>
static int launch_fdm(const FdmArgs& f, hipStream_t s) {
  constexpr int lds = fdm_lds_bytes<T>(MP, MODE, SPLIT);
  static_assert(lds <= 160 * 1024, "contraction tables exceed LDS");
  static DeviceCache cache;
  int dev = 0;
  if (int rc = current_device(&dev)) return rc;
  int resident = cache.v[dev].load(std::memory_order_relaxed);
  if (resident == 0) {
    int cus = 0, per_cu = 0, rc = CHEB_OK;
    if (lds > 64 * 1024)
      rc = hip_check(hipFuncSetAttribute((const void*)k_fdm_wave<T, MP, MODE, SPLIT>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, lds),
                     "contraction LDS attribute");
    if (!rc) rc = hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "CU count");
    if (!rc)
      rc = hip_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_fdm_wave<T, MP, MODE, SPLIT>,
                                                                  64 * kFdmWaves, lds),
                     "occupancy query");
    if (rc) return rc;
    resident = (cus > 0 ? cus : 1) * (per_cu > 0 ? per_cu : 1);
    cache.v[dev].store(resident, std::memory_order_relaxed);
  }
  const long long npen = (long long)f.m0 * f.m1 * f.m2 / f.m * f.nb;
  const long long wgs = ((npen + 15) / 16 + kFdmWaves - 1) / kFdmWaves;
  const int grid = (int)(wgs < resident ? (wgs > 0 ? wgs : 1) : resident);
  hipLaunchKernelGGL((k_fdm_wave<T, MP, MODE, SPLIT>), dim3(grid), dim3(64 * kFdmWaves), lds, s, f);
  return hip_check(hipGetLastError(), "axis contraction");
}

template <typename T, int MODE, int SPLIT>
static int launch_fdm_mode(const FdmArgs& f, hipStream_t s) {
  if constexpr (SPLIT != 0) {
    // only the widths whose halves are whole 16-row blocks
    switch ((f.m + 15) / 16) {
      case 2: return launch_fdm<T, 32, MODE, SPLIT>(f, s);
      case 4: return launch_fdm<T, 64, MODE, SPLIT>(f, s);
      case 6: return launch_fdm<T, 96, MODE, SPLIT>(f, s);
      case 8: return launch_fdm<T, 128, MODE, SPLIT>(f, s);
      default: set_error("even-odd contraction: unsupported width"); return CHEB_ERR_INVALID_ARG;
    }
  } else {
    switch ((f.m + 15) / 16) {
      case 1: return launch_fdm<T, 16, MODE, 0>(f, s);
      case 2: return launch_fdm<T, 32, MODE, 0>(f, s);
      case 3: return launch_fdm<T, 48, MODE, 0>(f, s);
      case 4: return launch_fdm<T, 64, MODE, 0>(f, s);
      case 5: return launch_fdm<T, 80, MODE, 0>(f, s);
      case 6: return launch_fdm<T, 96, MODE, 0>(f, s);
      case 7: return launch_fdm<T, 112, MODE, 0>(f, s);
      default: return launch_fdm<T, 128, MODE, 0>(f, s);
    }
  }
}

// split: 0 plain, 1 input through Q^T (the V^{-1} side), 2 output through Q
// (the V side), 3 the middle pair on a split axis; see k_fdm_wave
template <typename T>
static int launch_fdm_m(const FdmArgs& f, int mode, int split, hipStream_t s) {
  if (mode == (FDM_MID | FDM_SCALE)) {
    if (split == 3) return launch_fdm_mode<T, FDM_MID | FDM_SCALE, 3>(f, s);
    if constexpr (sizeof(T) == sizeof(float)) return launch_fdm_mode<T, FDM_MID | FDM_SCALE, 0>(f, s);
    set_error("middle pair: FP64 needs a split axis");
    return CHEB_ERR_INVALID_ARG;
  }
  if (split == 1) {
    switch (mode) {
      case FDM_XFULL: return launch_fdm_mode<T, FDM_XFULL, 1>(f, s);
      case FDM_SCALE: return launch_fdm_mode<T, FDM_SCALE, 1>(f, s);
      default: return launch_fdm_mode<T, 0, 1>(f, s);
    }
  }
  if (split == 2) {
    if (mode == FDM_YFULL) return launch_fdm_mode<T, FDM_YFULL, 2>(f, s);
    return launch_fdm_mode<T, 0, 2>(f, s);
  }
  switch (mode) {
    case FDM_XFULL: return launch_fdm_mode<T, FDM_XFULL, 0>(f, s);
    case FDM_YFULL: return launch_fdm_mode<T, FDM_YFULL, 0>(f, s);
    case FDM_SCALE: return launch_fdm_mode<T, FDM_SCALE, 0>(f, s);
    default: return launch_fdm_mode<T, 0, 0>(f, s);
  }
}

// fragment table of axis a for side dir (0: the V^{-1} side, 1: the V side)
// and the transposed preconditioner (tr)
template <typename T>
static const T* fdm_tab(const cheb_plan* p, int a, int dir, bool tr) {
  return pc_base<T>(p) + p->pc_ax[a].off_tab[dir][tr ? 1 : 0];
}

// Y = (side dir of axis a) applied along `axis` of the packed block X (m0, m1,
// m2): V^{-1} (dir 0) or V (dir 1), transposed with tr.  nb consecutive blocks
// of the same shape are contracted by one launch.
template <typename T>
static int axis_contract(const cheb_plan* p, int a, int dir, bool tr, const int* m, const T* X, T* Y,
                         hipStream_t s, int nb = 1) {
  if (m[a] <= 128) {
    FdmArgs f{};
    f.tab = fdm_tab<T>(p, a, dir, tr);
    f.X = X;
    f.Y = Y;
    f.m = m[a];
    f.axis = a;
    f.nb = nb;
    f.m0 = m[0];
    f.m1 = m[1];
    f.m2 = m[2];
    return launch_fdm_m<T>(f, 0, p->pc_ax[a].split ? dir + 1 : 0, s);
  }
  const T* base = pc_base<T>(p);
  const T* M = base + ((dir == 0) != tr ? p->pc_ax[a].off_Vi : p->pc_ax[a].off_V);
  GemmArgs g;
  const long long msz = m[a];
  const long long ms_i = tr ? 1 : msz, ms_k = tr ? msz : 1;  // M(i,k) strides
  // centro-symmetric axis with halves in whole 16-row blocks: the split
  // contraction (V^{-1} side through Q^T, V side through Q; also transposed)
  const int ps = (m[a] + 1) / 2;
  const int kind = p->pc_ax[a].centro && ps % 16 == 0 ? dir + 1 : 0;
  g.ps = ps;
  if (a == 2) {
    // Y[r, i] = sum_k X[r, k] M[i, k]: rows r, columns i
    g.A = X; g.B = M; g.D = Y;
    g.I = m[0] * m[1] * nb; g.Kd = m[2]; g.C = m[2];
    g.a_si = m[2]; g.a_sk = 1;
    g.b_sk = ms_k; g.b_sc = ms_i;
    g.d_si = m[2]; g.d_sc = 1;
    g.a_sb = g.b_sb = g.d_sb = 0;
    if (kind == 0 || ps % kGt == 0) {
      dim3 grid((g.I + kGt - 1) / kGt, ((kind == 2 ? ps : g.C) + kGt - 1) / kGt, 1);
      if (kind == 1) hipLaunchKernelGGL((k_axis_gemm_lds<T, 1, true>), grid, dim3(256), 0, s, g);
      else if (kind == 2) hipLaunchKernelGGL((k_axis_gemm_lds<T, 2, true>), grid, dim3(256), 0, s, g);
      else hipLaunchKernelGGL((k_axis_gemm_lds<T, 0, true>), grid, dim3(256), 0, s, g);
    } else {
      dim3 grid((g.I + 15) / 16, ((kind == 2 ? ps : g.C) + 255) / 256, 1);
      if (kind == 1) hipLaunchKernelGGL((k_axis_gemm_split<T, 1, true>), grid, dim3(256), 0, s, g);
      else hipLaunchKernelGGL((k_axis_gemm_split<T, 2, true>), grid, dim3(256), 0, s, g);
    }
  } else {
    // Y_b = M X_b with X_b (m_axis x C), C = product of the later dims
    const int C = a == 0 ? m[1] * m[2] : m[2];
    const int batch = (a == 0 ? 1 : m[0]) * nb;
    g.A = M; g.B = X; g.D = Y;
    g.I = m[a]; g.Kd = m[a]; g.C = C;
    g.a_si = ms_i; g.a_sk = ms_k;
    g.b_sk = C; g.b_sc = 1;
    g.d_si = C; g.d_sc = 1;
    g.a_sb = 0;
    g.b_sb = g.d_sb = (long long)m[a] * C;
    if (kind == 0 || ps % kGt == 0) {
      dim3 grid(((kind == 2 ? ps : g.I) + kGt - 1) / kGt, (C + kGt - 1) / kGt, batch);
      if (kind == 1) hipLaunchKernelGGL((k_axis_gemm_lds<T, 1, false>), grid, dim3(256), 0, s, g);
      else if (kind == 2) hipLaunchKernelGGL((k_axis_gemm_lds<T, 2, false>), grid, dim3(256), 0, s, g);
      else hipLaunchKernelGGL((k_axis_gemm_lds<T, 0, false>), grid, dim3(256), 0, s, g);
    } else {
      dim3 grid(((kind == 2 ? ps : g.I) + 15) / 16, (C + 255) / 256, batch);
      if (kind == 1) hipLaunchKernelGGL((k_axis_gemm_split<T, 1, false>), grid, dim3(256), 0, s, g);
      else hipLaunchKernelGGL((k_axis_gemm_split<T, 2, false>), grid, dim3(256), 0, s, g);
    }
  }
  return hip_check(hipGetLastError(), "axis contraction");
}

// the fused path: every axis on the per-wave kernel, element offsets in the
// packed blocks below 2^31
static bool fused_ok(const int* m, int nb) {
  const size_t lim = (size_t)1 << 31;
  return m[0] <= 128 && m[1] <= 128 && m[2] <= 128 && (size_t)m[0] * m[1] * m[2] * (size_t)nb < lim;
}

// The six contractions on the matrix cores with the packing, the eigenvalue
// scaling and the unpacking folded into the first, the middle and the last
// (every axis with m <= 128); nb fields at offs (null: one field).  The last
// contraction also zeroes the boundary nodes of the output.
template <typename T>
static int precond_fused(const cheb_plan* p, const T* in, T* out, T* bufA, T* bufB, bool transpose, int nb,
                         const long long* offs, double inv_k, const int* sys, const double* kc, hipStream_t s) {
  const int n0 = p->g.n[0], n1 = p->g.n[1], n2 = p->g.n[2];
  const int m[3] = {n0 - 2, n1 - 2, n2 - 2};
  const T* base = pc_base<T>(p);
  auto run = [&](int a, int dir, const T* X, T* Y, int mode) {
    FdmArgs f{};
    f.gate = offs ? nullptr : p->gate;
    f.tab = fdm_tab<T>(p, a, dir, transpose);
    f.tab2 = fdm_tab<T>(p, a, 1, transpose);  // the middle pair's second contraction
    f.X = X;
    f.Y = Y;
    f.m = m[a];
    f.axis = a;
    f.nb = nb;
    f.m0 = m[0];
    f.m1 = m[1];
    f.m2 = m[2];
    f.offs = offs;
    if (mode & FDM_SCALE) {
      f.lam0 = base + p->pc_ax[0].off_lam;
      f.lam1 = base + p->pc_ax[1].off_lam;
      f.lam2 = base + p->pc_ax[2].off_lam;
      f.inv_k = inv_k;
      f.sys = sys;
      f.kc = kc;
    }
    const int split = p->pc_ax[a].split ? (mode & FDM_MID ? 3 : dir + 1) : 0;
    return launch_fdm_m<T>(f, mode, split, s);
  };
  int rc = run(0, 0, in, bufA, FDM_XFULL);
  // the two z contractions and the scaling between them as one kernel where
  // both tables fit in LDS (FP64: split axes only)
  const bool mid = p->pc_ax[2].split || sizeof(T) == sizeof(float);
  if (!rc) rc = run(1, 0, bufA, bufB, 0);
  if (mid) {
    if (!rc) rc = run(2, 0, bufB, bufA, FDM_MID | FDM_SCALE);
  } else {
    if (!rc) rc = run(2, 0, bufB, bufA, FDM_SCALE);
    if (!rc) rc = run(2, 1, bufA, bufB, 0);
    std::swap(bufA, bufB);
  }
  if (!rc) rc = run(1, 1, bufA, bufB, 0);
  if (!rc) rc = run(0, 1, bufB, out, FDM_YFULL);  // also zeroes the boundary nodes of out
  return rc;
}

template <typename T>
int precond_apply(const cheb_plan* p, const T* in, T* out, T* bufA, T* bufB, double kc, bool transpose,
                  hipStream_t s) {
  const int n0 = p->g.n[0], n1 = p->g.n[1], n2 = p->g.n[2];
  const int m[3] = {n0 - 2, n1 - 2, n2 - 2};
  if (fused_ok(m, 1))
    return precond_fused<T>(p, in, out, bufA, bufB, transpose, 1, nullptr, 1.0 / kc, nullptr, nullptr, s);
  const size_t tot = (size_t)m[0] * m[1] * m[2];
  const T* base = pc_base<T>(p);
  hipLaunchKernelGGL(k_pack_interior<T>, dim3(grid1(tot)), dim3(256), 0, s, in, bufA, n0, n1, n2);
  int rc = hip_check(hipGetLastError(), "pack");
  if (rc) return rc;
  // forward: V^{-1} (or V^T for the transpose) along x, y, z
  T* x = bufA;
  T* y = bufB;
  for (int a = 0; a < 3 && !rc; ++a) {
    rc = axis_contract<T>(p, a, 0, transpose, m, x, y, s);
    std::swap(x, y);
  }
  if (rc) return rc;
  hipLaunchKernelGGL(k_eig_scale<T>, dim3(grid1(tot)), dim3(256), 0, s, x, base + p->pc_ax[0].off_lam,
                     base + p->pc_ax[1].off_lam, base + p->pc_ax[2].off_lam, 1.0 / kc, m[0], m[1], m[2]);
  rc = hip_check(hipGetLastError(), "eigen scale");
  for (int a = 2; a >= 0 && !rc; --a) {
    rc = axis_contract<T>(p, a, 1, transpose, m, x, y, s);
    std::swap(x, y);
  }
  if (rc) return rc;
  hipLaunchKernelGGL(k_unpack_interior<T>, dim3(grid1((size_t)n0 * n1 * n2)), dim3(256), 0, s, x, out, n0, n1, n2);
  return hip_check(hipGetLastError(), "unpack");
}

// plain GEMM on the matrix cores, exposed for the layout test:
// D (I x C) = A (I x K) B (K x C), all row-major
template <typename T>
int mfma_gemm(const T* A, const T* B, T* D, int I, int K, int C, hipStream_t s) {
  GemmArgs g;
  g.A = A; g.B = B; g.D = D;
  g.I = I; g.Kd = K; g.C = C;
  g.a_si = K; g.a_sk = 1; g.b_sk = C; g.b_sc = 1; g.d_si = C; g.d_sc = 1;
  g.a_sb = g.b_sb = g.d_sb = 0;
  dim3 grid((I + 15) / 16, (C + 255) / 256, 1);
  hipLaunchKernelGGL(k_axis_gemm<T>, grid, dim3(256), 0, s, g);
  return hip_check(hipGetLastError(), "mfma gemm");
}

template <typename T>
int precond_apply_batch(const cheb_plan* rep, const T* in, T* out, const long long* offs, const int* sys,
                        const double* kc, int nmem, size_t span, T* bufA, T* bufB, hipStream_t s) {
  if (nmem <= 0) return CHEB_OK;
  const int n0 = rep->g.n[0], n1 = rep->g.n[1], n2 = rep->g.n[2];
  const int m[3] = {n0 - 2, n1 - 2, n2 - 2};
  (void)span;
  if (fused_ok(m, nmem))
    return precond_fused<T>(rep, in, out, bufA, bufB, false, nmem, offs, 0.0, sys, kc, s);
  const size_t tot = (size_t)m[0] * m[1] * m[2];
  const T* base = pc_base<T>(rep);
  hipLaunchKernelGGL(k_pack_interior_b<T>, dim3(grid1(tot), nmem), dim3(256), 0, s, in, offs, bufA, n0, n1, n2);
  int rc = hip_check(hipGetLastError(), "batched pack");
  T* x = bufA;
  T* y = bufB;
  for (int a = 0; a < 3 && !rc; ++a) {
    rc = axis_contract<T>(rep, a, 0, false, m, x, y, s, nmem);
    std::swap(x, y);
  }
  if (rc) return rc;
  hipLaunchKernelGGL(k_eig_scale_b<T>, dim3(grid1(tot), nmem), dim3(256), 0, s, x, base + rep->pc_ax[0].off_lam,
                     base + rep->pc_ax[1].off_lam, base + rep->pc_ax[2].off_lam, sys, kc, m[0], m[1], m[2]);
  rc = hip_check(hipGetLastError(), "batched eigen scale");
  for (int a = 2; a >= 0 && !rc; --a) {
    rc = axis_contract<T>(rep, a, 1, false, m, x, y, s, nmem);
    std::swap(x, y);
  }
  if (rc) return rc;
  hipLaunchKernelGGL(k_unpack_interior_b<T>, dim3(grid1((size_t)n0 * n1 * n2), nmem), dim3(256), 0, s, x, offs,
                     out, n0, n1, n2);
  return hip_check(hipGetLastError(), "batched unpack");
}

template int precond_apply_batch<double>(const cheb_plan*, const double*, double*, const long long*, const int*,
                                         const double*, int, size_t, double*, double*, hipStream_t);
template int precond_apply_batch<float>(const cheb_plan*, const float*, float*, const long long*, const int*,
                                        const double*, int, size_t, float*, float*, hipStream_t);
template int precond_apply<double>(const cheb_plan*, const double*, double*, double*, double*, double, bool,
                                   hipStream_t);
template int precond_apply<float>(const cheb_plan*, const float*, float*, float*, float*, double, bool,
                                  hipStream_t);
template int mfma_gemm<double>(const double*, const double*, double*, int, int, int, hipStream_t);
template int mfma_gemm<float>(const float*, const float*, float*, int, int, int, hipStream_t);

}  // namespace cheb

using namespace cheb;

extern "C" int cheb_debug_gemm(int32_t precision, const void* A, const void* B, void* D, int32_t I, int32_t K,
                               int32_t C, void* stream) {
  if (!A || !B || !D || I <= 0 || K <= 0 || C <= 0) {
    set_error("invalid argument");
    return CHEB_ERR_INVALID_ARG;
  }
  if (precision == CHEB_F32)
    return mfma_gemm<float>((const float*)A, (const float*)B, (float*)D, I, K, C, (hipStream_t)stream);
  return mfma_gemm<double>((const double*)A, (const double*)B, (double*)D, I, K, C, (hipStream_t)stream);
}

extern "C" int cheb_precond_apply(cheb_plan* plan, int32_t field_precision, double kc, const void* in, void* out,
                                  uint32_t flags) {
  if (!plan || !in || !out) {
    set_error("null argument");
    return CHEB_ERR_INVALID_ARG;
  }
  if (field_precision != CHEB_F64 && field_precision != CHEB_F32) {
    set_error("preconditioner: field_precision must be CHEB_F64 or CHEB_F32");
    return CHEB_ERR_INVALID_ARG;
  }
  if ((flags & ~(uint32_t)CHEB_APPLY_TRANSPOSE) != 0) {
    set_error("preconditioner: flags must be 0 or CHEB_APPLY_TRANSPOSE");
    return CHEB_ERR_INVALID_ARG;
  }
  if (!(kc > 0.0) || !std::isfinite(kc)) {
    set_error("preconditioner: kc must be positive and finite");
    return CHEB_ERR_INVALID_ARG;
  }
  const size_t es = field_precision == CHEB_F64 ? sizeof(double) : sizeof(float);
  const size_t pb = round_up((size_t)(plan->g.n[0] - 2) * (plan->g.n[1] - 2) * (plan->g.n[2] - 2) * es, 256);
  if (!plan->ws || plan->ws_bytes < 2 * pb) {
    set_error("preconditioner: the workspace must hold two interior blocks");
    return CHEB_ERR_WORKSPACE;
  }
  int rc = precond_setup(plan);
  if (rc) return rc;
  // outside a solve nothing gates the contractions
  const int* gate = plan->gate;
  plan->gate = nullptr;
  char* w = (char*)plan->ws;
  const bool tr = (flags & CHEB_APPLY_TRANSPOSE) != 0;
  if (field_precision == CHEB_F64)
    rc = precond_apply<double>(plan, (const double*)in, (double*)out, (double*)w, (double*)(w + pb), kc, tr,
                               plan->stream);
  else
    rc = precond_apply<float>(plan, (const float*)in, (float*)out, (float*)w, (float*)(w + pb), kc, tr,
                              plan->stream);
  plan->gate = gate;
  return rc;
}
