// Boundary elimination on the full nodal state (Section 2.3.1):
//   lift:       x_r = G x_k + H g  -- Dirichlet nodes take their data, then the
//               Neumann-owned end values of the pencils along z, y and x solve
//               their 1x1 or 2x2 block of B_r with the pencil's other values;
//   transpose:  the homogeneous lift transposed, steps in reverse order (x, y,
//               z), each adding the end value (mapped by the transposed block)
//               onto the pencil's other values; finally boundary entries are 0.
// The lift reads each pencil with many lanes (a wave per z pencil; eight waves
// per 64 x or y pencils); the transpose runs one thread per pencil.
#include "internal.h"
#include "pencil.h"

namespace cheb {

namespace {

// owner face of node (i, j, k): lowest-axis Dirichlet face containing it, else
// lowest-axis Neumann face, -1 for interior nodes
__device__ int node_owner(int i, int j, int k, const int* n, const int* bc) {
  const int idx[3] = {i, j, k};
  int own = -1;
  for (int pass = 0; pass < 2 && own < 0; ++pass) {
    for (int a = 0; a < 3 && own < 0; ++a) {
      int f = -1;
      if (idx[a] == 0) f = 2 * a;
      else if (idx[a] == n[a] - 1) f = 2 * a + 1;
      if (f >= 0 && bc[f] == pass) own = f;
    }
  }
  return own;
}

struct LiftArgs {
  int n[3];
  int bc[6];
  int bcmask;
  long long goff[6];
  const double* rn;  // per-node Robin coefficients (packed like g) or null
};

// the end block's diagonal entries of pencil p along `axis` with its own
// nodes' Robin coefficients
__device__ inline void node_block(const LiftArgs& a, int axis, int p, double& m00, double& mNN) {
  if (a.rn) {
    m00 -= a.rn[a.goff[2 * axis] + p];
    mNN += a.rn[a.goff[2 * axis + 1] + p];
  }
}

template <typename T>
__global__ void k_set_dirichlet(T* U, const T* g, int f, LiftArgs a) {
  const int ax = f / 2, side = f % 2;
  const int tb = ax == 0 ? 1 : 0, tc = ax == 2 ? 1 : 2;
  const int nb = a.n[tb], nc = a.n[tc];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nb * nc) return;
  const int ib = t / nc, ic = t - ib * nc;
  int idx[3];
  idx[ax] = side ? a.n[ax] - 1 : 0;
  idx[tb] = ib;
  idx[tc] = ic;
  if (node_owner(idx[0], idx[1], idx[2], a.n, a.bc) != f) return;
  const size_t ad = ((size_t)idx[0] * a.n[1] + idx[1]) * a.n[2] + idx[2];
  U[ad] = g ? g[a.goff[f] + t] : T(0);
}

// Pencils along x or y: lanes take adjacent pencils (adjacent addresses, so
// every load is coalesced) and the 8 waves of a workgroup split each pencil's
// inner nodes, so a launch holds eight times as many waves as pencils/64; the
// partial row sums meet in LDS and wave 0 solves for the end values.
template <typename T>
__global__ __launch_bounds__(512) void k_lift_axis(T* U, const T* g, int axis, const T* drow0, const T* drowN,
                                                   double m00, double m0N, double mN0, double mNN, LiftArgs a) {
  __shared__ double red[2][8][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int p = blockIdx.x * 64 + lane;
  const int np = pencil_count(axis, a.n);
  long long base = 0;
  const int fl = p < np ? pencil_flags(axis, p, np, a.n[0], a.n[1], a.n[2], a.bcmask, &base) : 0;
  const bool nlo = (fl & PF_VALID) && (fl & PF_OWN_LO) && a.bc[2 * axis] == 1;
  const bool nhi = (fl & PF_VALID) && (fl & PF_OWN_HI) && a.bc[2 * axis + 1] == 1;
  const long long st = pencil_stride(axis, a.n);
  const int N = a.n[axis] - 1;
  T* u = U + base;
  double s0 = 0.0, sN = 0.0;
  if (nlo || nhi) {
    for (int m = 1 + w; m < N; m += 8) {
      const double v = double(u[m * st]);
      s0 = fma(double(drow0[m]), v, s0);
      sN = fma(double(drowN[m]), v, sN);
    }
  }
  red[0][w][lane] = s0;
  red[1][w][lane] = sN;
  __syncthreads();
  if (w != 0 || !(nlo || nhi)) return;
  s0 = 0.0;
  sN = 0.0;
  for (int k = 0; k < 8; ++k) {
    s0 += red[0][k][lane];
    sN += red[1][k][lane];
  }
  const double glo = g ? double(g[a.goff[2 * axis] + p]) : 0.0;
  const double ghi = g ? double(g[a.goff[2 * axis + 1] + p]) : 0.0;
  node_block(a, axis, p, m00, mNN);
  if (nlo && nhi) {
    const double r0 = -glo - s0, rN = ghi - sN;
    const double det = m00 * mNN - m0N * mN0;
    u[0] = T((r0 * mNN - m0N * rN) / det);
    u[N * st] = T((m00 * rN - mN0 * r0) / det);
  } else if (nlo) {
    const double r0 = -glo - s0 - double(drow0[N]) * double(u[N * st]);
    u[0] = T(r0 / m00);
  } else {
    const double rN = ghi - sN - double(drowN[0]) * double(u[0]);
    u[N * st] = T(rN / mNN);
  }
}

// The same lift for pencils along z, whose nodes are contiguous: one 64-lane
// wave per pencil reads it in coalesced strips, the two row sums are reduced
// across the wave, and lane 0 solves for the end values (one thread per pencil
// would read 64 separate lines per load here).
template <typename T>
__global__ __launch_bounds__(256) void k_lift_z_wave(T* U, const T* g, const T* drow0, const T* drowN, double m00,
                                                     double m0N, double mN0, double mNN, LiftArgs a) {
  const int lane = threadIdx.x & 63;
  const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int np = pencil_count(2, a.n);
  if (p >= np) return;  // uniform per wave
  long long base;
  const int fl = pencil_flags(2, p, np, a.n[0], a.n[1], a.n[2], a.bcmask, &base);
  if (!(fl & PF_VALID)) return;
  const bool nlo = (fl & PF_OWN_LO) && a.bc[4] == 1;
  const bool nhi = (fl & PF_OWN_HI) && a.bc[5] == 1;
  if (!nlo && !nhi) return;
  const int N = a.n[2] - 1;
  T* u = U + base;
  double s0 = 0.0, sN = 0.0;
  for (int m = 1 + lane; m < N; m += 64) {
    const double v = double(u[m]);
    s0 = fma(double(drow0[m]), v, s0);
    sN = fma(double(drowN[m]), v, sN);
  }
  for (int o = 32; o > 0; o >>= 1) {
    s0 += __shfl_xor(s0, o);
    sN += __shfl_xor(sN, o);
  }
  if (lane != 0) return;
  const double glo = g ? double(g[a.goff[4] + p]) : 0.0;
  const double ghi = g ? double(g[a.goff[5] + p]) : 0.0;
  node_block(a, 2, p, m00, mNN);
  if (nlo && nhi) {
    const double r0 = -glo - s0, rN = ghi - sN;
    const double det = m00 * mNN - m0N * mN0;
    u[0] = T((r0 * mNN - m0N * rN) / det);
    u[N] = T((m00 * rN - mN0 * r0) / det);
  } else if (nlo) {
    const double r0 = -glo - s0 - double(drow0[N]) * double(u[N]);
    u[0] = T(r0 / m00);
  } else {
    const double rN = ghi - sN - double(drowN[0]) * double(u[0]);
    u[N] = T(rN / mNN);
  }
}

template <typename T>
__global__ void k_lift_t_axis(T* W, int axis, const T* drow0, const T* drowN, double m00, double m0N,
                              double mN0, double mNN, LiftArgs a) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int np = pencil_count(axis, a.n);
  long long base;
  const int fl = pencil_flags(axis, p, np, a.n[0], a.n[1], a.n[2], a.bcmask, &base);
  if (!(fl & PF_VALID)) return;
  const bool nlo = (fl & PF_OWN_LO) && a.bc[2 * axis] == 1;
  const bool nhi = (fl & PF_OWN_HI) && a.bc[2 * axis + 1] == 1;
  if (!nlo && !nhi) return;
  const long long st = pencil_stride(axis, a.n);
  const int N = a.n[axis] - 1;
  T* w = W + base;
  const double z0 = double(w[0]), zN = double(w[N * st]);
  double mu0 = 0.0, muN = 0.0;
  int m_lo = 1, m_hi = N - 1;
  node_block(a, axis, p, m00, mNN);
  if (nlo && nhi) {
    const double det = m00 * mNN - m0N * mN0;
    mu0 = (z0 * mNN - zN * mN0) / det;
    muN = (zN * m00 - z0 * m0N) / det;
  } else if (nlo) {
    mu0 = z0 / m00;
    m_hi = N;
  } else {
    muN = zN / mNN;
    m_lo = 0;
  }
  for (int m = m_lo; m <= m_hi; ++m) {
    const double v = double(w[m * st]) - mu0 * double(drow0[m]) - muN * double(drowN[m]);
    w[m * st] = T(v);
  }
  if (nlo) w[0] = T(0);
  if (nhi) w[N * st] = T(0);
}

LiftArgs make_args(const cheb_plan* p) {
  LiftArgs a;
  long long off = 0;
  for (int i = 0; i < 3; ++i) a.n[i] = p->g.n[i];
  a.bcmask = bc_mask(p->g.bc);
  for (int f = 0; f < 6; ++f) {
    a.bc[f] = p->g.bc[f];
    a.goff[f] = off;
    const int ax = f / 2;
    const int tb = ax == 0 ? 1 : 0, tc = ax == 2 ? 1 : 2;
    off += (long long)p->g.n[tb] * p->g.n[tc];
  }
  a.rn = p->rn64;
  return a;
}

template <typename T>
const T* plan_rows(const cheb_plan* p, int a, int s);
template <>
const double* plan_rows<double>(const cheb_plan* p, int a, int s) { return dconst64(p, a, s); }
template <>
const float* plan_rows<float>(const cheb_plan* p, int a, int s) { return dconst32(p, a, s); }

}  // namespace

template <typename T>
int lift_full(const cheb_plan* p, T* U, const T* g_faces, hipStream_t s) {
  const LiftArgs a = make_args(p);
  for (int f = 0; f < 6; ++f) {
    if (p->g.bc[f] != 0) continue;
    const int ax = f / 2;
    const int tb = ax == 0 ? 1 : 0, tc = ax == 2 ? 1 : 2;
    const int cnt = p->g.n[tb] * p->g.n[tc];
    hipLaunchKernelGGL(k_set_dirichlet<T>, dim3((cnt + 255) / 256), dim3(256), 0, s, U, g_faces, f, a);
  }
  for (int ax = 2; ax >= 0; --ax) {
    if (p->g.bc[2 * ax] != 1 && p->g.bc[2 * ax + 1] != 1) continue;
    const int np = pencil_count(ax, a.n);
    const AxisConst& c = p->ax[ax];
    if (ax == 2)
      hipLaunchKernelGGL(k_lift_z_wave<T>, dim3((np + 3) / 4), dim3(256), 0, s, U, g_faces, plan_rows<T>(p, ax, 0),
                         plan_rows<T>(p, ax, 1), c.m00, c.m0N, c.mN0, c.mNN, a);
    else
      hipLaunchKernelGGL(k_lift_axis<T>, dim3((np + 63) / 64), dim3(512), 0, s, U, g_faces, ax,
                         plan_rows<T>(p, ax, 0), plan_rows<T>(p, ax, 1), c.m00, c.m0N, c.mN0, c.mNN, a);
  }
  return hip_check(hipGetLastError(), "lift_full");
}

template <typename T>
int lift_transpose(const cheb_plan* p, T* W, hipStream_t s) {
  const LiftArgs a = make_args(p);
  for (int ax = 0; ax < 3; ++ax) {
    if (p->g.bc[2 * ax] != 1 && p->g.bc[2 * ax + 1] != 1) continue;
    const int np = pencil_count(ax, a.n);
    const AxisConst& c = p->ax[ax];
    hipLaunchKernelGGL(k_lift_t_axis<T>, dim3((np + 127) / 128), dim3(128), 0, s, W, ax,
                       plan_rows<T>(p, ax, 0), plan_rows<T>(p, ax, 1), c.m00, c.m0N, c.mN0, c.mNN, a);
  }
  int rc = hip_check(hipGetLastError(), "lift_transpose");
  if (rc) return rc;
  return mask_interior<T>(W, p->g.n, s);
}

template int lift_full<double>(const cheb_plan*, double*, const double*, hipStream_t);
template int lift_full<float>(const cheb_plan*, float*, const float*, hipStream_t);
template int lift_transpose<double>(const cheb_plan*, double*, hipStream_t);
template int lift_transpose<float>(const cheb_plan*, float*, hipStream_t);

}  // namespace cheb
