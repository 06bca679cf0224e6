// C ABI: plans, operator application, derivatives, volume averages, status.
// The solver entry points live in solver.hip, prolongation in prolong.hip.
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "internal.h"
#include "pencil.h"

namespace cheb {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return CHEB_OK;
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return CHEB_ERR_DEVICE;
}

namespace {

// Boundary rows of the ascending, scaled differentiation matrix, from the
// closed forms of the endpoint rows of the CGL differentiation matrix
// (descending nodes: D_00 = (2N^2+1)/6, D_0j = (-1)^j / sin^2(pi j / 2N),
// D_0N = (-1)^N / 2; ascending order negates, and row N follows from the
// centro-antisymmetry).
void boundary_rows(int N, double L, std::vector<double>& r0, std::vector<double>& rN) {
  r0.assign(N + 1, 0.0);
  rN.assign(N + 1, 0.0);
  const double s = 2.0 / L;
  const double corner = (2.0 * N * N + 1.0) / 6.0;
  const double half = (N % 2 == 0) ? 0.5 : -0.5;  // (-1)^N / 2
  for (int j = 1; j < N; ++j) {
    const double sj = std::sin(M_PI * j / (2.0 * N));
    const double dj = ((j % 2 == 0) ? 1.0 : -1.0) / (sj * sj);  // descending D_0j
    const int k = N - j;
    const double sk = std::sin(M_PI * k / (2.0 * N));
    const double dk = ((k % 2 == 0) ? 1.0 : -1.0) / (sk * sk);  // descending D_0k
    r0[j] = -dj * s;
    rN[j] = dk * s;
  }
  r0[0] = -corner * s;
  r0[N] = -half * s;
  rN[0] = half * s;
  rN[N] = corner * s;
}

// Clenshaw-Curtis weights on [0, L] (closed form, Waldvogel / Trefethen).
void cc_weights(int N, double L, std::vector<double>& w) {
  w.assign(N + 1, 0.0);
  std::vector<double> v(N + 1, 1.0);
  const bool even = (N % 2 == 0);
  const double wend = even ? 1.0 / (double(N) * N - 1.0) : 1.0 / (double(N) * N);
  for (int j = 1; j < N; ++j) {
    const double th = M_PI * j / N;
    double t = 1.0;
    const int kmax = even ? N / 2 - 1 : (N - 1) / 2;
    for (int k = 1; k <= kmax; ++k) t -= 2.0 * std::cos(2.0 * k * th) / (4.0 * k * k - 1.0);
    if (even) t -= std::cos(N * th) / (double(N) * N - 1.0);
    w[j] = 2.0 * t / N;
  }
  w[0] = w[N] = wend;
  for (double& x : w) x *= L / 2.0;
}

}  // namespace
}  // namespace cheb

using namespace cheb;

namespace {

// Time one reduced apply configuration: 2 warm-up applies, then `reps` timed
// with events on the plan's stream; returns microseconds per apply.
template <typename T>
static int time_apply(cheb_plan* p, const T* K, const T* u, T* y, int reps, double* us) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = hip_check(hipEventCreate(&e0), "hipEventCreate");
  if (!rc) rc = hip_check(hipEventCreate(&e1), "hipEventCreate");
  for (int i = 0; !rc && i < 2; ++i) rc = apply_t<T>(p, K, u, y, 1, p->stream);
  if (!rc) rc = hip_check(hipEventRecord(e0, p->stream), "hipEventRecord");
  for (int i = 0; !rc && i < reps; ++i) rc = apply_t<T>(p, K, u, y, 1, p->stream);
  if (!rc) rc = hip_check(hipEventRecord(e1, p->stream), "hipEventRecord");
  if (!rc) rc = hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
  float ms = 0.f;
  if (!rc) rc = hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  *us = 1e3 * ms / reps;
  return rc;
}

template <typename T>
static int autotune_t(cheb_plan* p, const T* K, const T* u, T* y, double* report, int report_len) {
  const int pi = sizeof(T) == sizeof(double) ? 0 : 1;
  const int saved_route = p->route;
  int saved_var[3];
  for (int a = 0; a < 3; ++a) saved_var[a] = p->dense_var[a][pi];
  bool any = false;
  for (int a = 0; a < 3; ++a) any = any || p->dd_ok[a];
  double t[3] = {-1.0, -1.0, -1.0};  // FFT route, matrix route tile shape 0, tile shape 1
  int rc = CHEB_OK;
  p->route = CHEB_ROUTE_FFT;
  rc = time_apply<T>(p, K, u, y, 10, &t[0]);
  for (int v = 0; !rc && any && v < 2; ++v) {
    p->route = CHEB_ROUTE_MATRIX;
    for (int a = 0; a < 3; ++a) p->dense_var[a][pi] = v;
    rc = time_apply<T>(p, K, u, y, 10, &t[1 + v]);
  }
  p->route = saved_route;
  if (rc) {
    for (int a = 0; a < 3; ++a) p->dense_var[a][pi] = saved_var[a];
    return rc;
  }
  int best = 0;
  for (int c = 1; c < 3; ++c)
    if (t[c] >= 0.0 && t[c] < t[best]) best = c;
  p->auto_fft[pi] = best == 0;
  for (int a = 0; a < 3; ++a) p->dense_var[a][pi] = best == 0 ? saved_var[a] : best - 1;
  for (int c = 0; c < 3 && c < report_len; ++c) report[c] = t[c];
  if (report_len > 3) report[3] = best;
  return CHEB_OK;
}

}  // namespace

extern "C" {

const char* cheb_last_error(void) { return g_last_error.c_str(); }

const char* cheb_status_string(int status) {
  switch (status) {
    case CHEB_OK: return "ok";
    case CHEB_NOT_CONVERGED: return "not converged";
    case CHEB_STAGNATED: return "stagnated";
    case CHEB_ERR_INVALID_ARG: return "invalid argument";
    case CHEB_ERR_SINGULAR_BC: return "singular boundary conditions (all faces Neumann)";
    case CHEB_ERR_BAD_INPUT: return "bad input (NaN/Inf or non-positive conductivity)";
    case CHEB_ERR_DEVICE: return "device error";
    case CHEB_ERR_WORKSPACE: return "workspace missing or too small";
    case CHEB_ERR_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

int cheb_plan_create(const cheb_grid* grid, int32_t precision, void* stream, cheb_plan** out) {
  if (!grid || !out) {
    set_error("null argument");
    return CHEB_ERR_INVALID_ARG;
  }
  *out = nullptr;
  for (int a = 0; a < 3; ++a) {
    if (grid->n[a] < 3 || grid->n[a] > 513) {
      set_error("grid size must be in [3, 513] on every axis");
      return CHEB_ERR_INVALID_ARG;
    }
    if (!(grid->hi[a] > grid->lo[a]) || !std::isfinite(grid->lo[a]) || !std::isfinite(grid->hi[a])) {
      set_error("need finite lo < hi on every axis");
      return CHEB_ERR_INVALID_ARG;
    }
  }
  bool allN = true, anyRobin = false;
  for (int f = 0; f < 6; ++f) {
    if (grid->bc[f] != CHEB_DIRICHLET && grid->bc[f] != CHEB_NEUMANN) {
      set_error("face type must be CHEB_DIRICHLET or CHEB_NEUMANN");
      return CHEB_ERR_INVALID_ARG;
    }
    if (!std::isfinite(grid->robin[f]) || (grid->bc[f] == CHEB_DIRICHLET && grid->robin[f] != 0.0)) {
      set_error("Robin coefficients must be finite, and 0 on Dirichlet faces");
      return CHEB_ERR_INVALID_ARG;
    }
    allN = allN && grid->bc[f] == CHEB_NEUMANN;
    anyRobin = anyRobin || grid->robin[f] != 0.0;
  }
  if (allN && !anyRobin) {
    set_error("all six faces Neumann: the problem is singular");
    return CHEB_ERR_SINGULAR_BC;
  }
  if (precision != CHEB_F64 && precision != CHEB_F32 && precision != CHEB_MIXED) {
    set_error("precision must be CHEB_F64, CHEB_F32 or CHEB_MIXED");
    return CHEB_ERR_INVALID_ARG;
  }
  cheb_plan* p = new (std::nothrow) cheb_plan();
  if (!p) {
    set_error("out of host memory");
    return CHEB_ERR_INVALID_ARG;
  }
  std::memset((void*)p, 0, sizeof(cheb_plan));
  p->g = *grid;
  p->prec = precision;
  p->stream = (hipStream_t)stream;
  p->npts = (size_t)grid->n[0] * grid->n[1] * grid->n[2];
  size_t nmax = 0;
  for (int a = 0; a < 3; ++a) {
    AxisConst& c = p->ax[a];
    c.N = grid->n[a] - 1;
    c.L = grid->hi[a] - grid->lo[a];
    c.cscale = -1.0 / (double(c.N) * c.L);
    if ((size_t)grid->n[a] > nmax) nmax = grid->n[a];
  }
  p->dconst_stride = round_up(nmax, 64);
  const size_t cnt = 3 * kConstSlots * p->dconst_stride;
  std::vector<double> h64(cnt, 0.0);
  std::vector<float> h32(cnt, 0.0f);
  for (int a = 0; a < 3; ++a) {
    AxisConst& c = p->ax[a];
    std::vector<double> r0, rN, w;
    boundary_rows(c.N, c.L, r0, rN);
    cc_weights(c.N, c.L, w);
    // end-value block of the boundary rows: lo row -(D u)_0 + sigma_lo u_0,
    // hi row (D u)_N + sigma_hi u_N (sigma = 0 on plain Neumann faces)
    c.m00 = r0[0] - grid->robin[2 * a];
    c.m0N = r0[c.N];
    c.mN0 = rN[0];
    c.mNN = rN[c.N] + grid->robin[2 * a + 1];
    const bool nlo = grid->bc[2 * a] == CHEB_NEUMANN, nhi = grid->bc[2 * a + 1] == CHEB_NEUMANN;
    const double det = c.m00 * c.mNN - c.m0N * c.mN0;
    const double scale = std::fabs(c.m00 * c.mNN) + std::fabs(c.m0N * c.mN0);
    if ((nlo && !(std::fabs(c.m00) > 1e-12 * std::fabs(r0[0]))) ||
        (nhi && !(std::fabs(c.mNN) > 1e-12 * std::fabs(rN[c.N]))) ||
        (nlo && nhi && !(std::fabs(det) > 1e-12 * scale))) {
      set_error("Robin coefficients make a boundary elimination block singular");
      delete p;
      return CHEB_ERR_INVALID_ARG;
    }
    for (int j = 0; j <= c.N; ++j) {
      h64[(kConstSlots * a + 0) * p->dconst_stride + j] = r0[j];
      h64[(kConstSlots * a + 1) * p->dconst_stride + j] = rN[j];
      h64[(kConstSlots * a + 2) * p->dconst_stride + j] = w[j];
    }
    // twiddles of the length-2N FFT of the even extension: W^j = exp(-i pi j / N)
    for (int j = 0; j < 2 * c.N; ++j) {
      h64[(kConstSlots * a + 3) * p->dconst_stride + 2 * j] = std::cos(M_PI * j / c.N);
      h64[(kConstSlots * a + 3) * p->dconst_stride + 2 * j + 1] = -std::sin(M_PI * j / c.N);
    }
  }
  for (size_t i = 0; i < cnt; ++i) h32[i] = float(h64[i]);
  if (hip_check(hipGetDevice(&p->device), "hipGetDevice")) {
    delete p;
    return CHEB_ERR_DEVICE;
  }
  int rc = hip_check(hipMalloc((void**)&p->dconst64, cnt * sizeof(double)), "hipMalloc(plan constants)");
  if (!rc) rc = hip_check(hipMalloc((void**)&p->dconst32, cnt * sizeof(float)), "hipMalloc(plan constants)");
  if (!rc)
    rc = hip_check(hipMemcpy(p->dconst64, h64.data(), cnt * sizeof(double), hipMemcpyHostToDevice),
                   "hipMemcpy(plan constants)");
  if (!rc)
    rc = hip_check(hipMemcpy(p->dconst32, h32.data(), cnt * sizeof(float), hipMemcpyHostToDevice),
                   "hipMemcpy(plan constants)");
  if (!rc) rc = dense_setup(p);
  p->hpinned_len = 4096;
  if (!rc)
    rc = hip_check(hipHostMalloc((void**)&p->hpinned, p->hpinned_len * sizeof(double), hipHostMallocDefault),
                   "hipHostMalloc");
  if (rc) {
    if (p->dconst64) (void)hipFree(p->dconst64);
    if (p->dconst32) (void)hipFree(p->dconst32);
    if (p->dd64) (void)hipFree(p->dd64);
    if (p->dd32) (void)hipFree(p->dd32);
    if (p->pair_buf) (void)hipFree(p->pair_buf);
    if (p->hpinned) (void)hipHostFree(p->hpinned);
    delete p;
    return rc;
  }
  *out = p;
  return CHEB_OK;
}

int cheb_plan_set_workspace(cheb_plan* plan, void* dev_ptr, size_t bytes) {
  if (!plan) {
    set_error("null plan");
    return CHEB_ERR_INVALID_ARG;
  }
  if (dev_ptr && ((uintptr_t)dev_ptr % 256) != 0) {
    set_error("workspace must be 256-byte aligned");
    return CHEB_ERR_WORKSPACE;
  }
  plan->ws = dev_ptr;
  plan->ws_bytes = dev_ptr ? bytes : 0;
  return CHEB_OK;
}

int cheb_plan_set_stream(cheb_plan* plan, void* stream) {
  if (!plan) {
    set_error("null plan");
    return CHEB_ERR_INVALID_ARG;
  }
  plan->stream = (hipStream_t)stream;
  return CHEB_OK;
}

static void drop_precond(cheb_plan* p) {
  if (p->pc64) (void)hipFree(p->pc64);
  if (p->pc32) (void)hipFree(p->pc32);
  p->pc64 = nullptr;
  p->pc32 = nullptr;
  p->pc_ready = 0;
}

int cheb_plan_set_robin_nodes(cheb_plan* plan, const double* sigma_faces) {
  if (!plan) {
    set_error("null plan");
    return CHEB_ERR_INVALID_ARG;
  }
  const int* n = plan->g.n;
  const size_t cnt = (size_t)face_offset(6, n);
  if (!sigma_faces) {
    if (plan->rn64) {
      int rc = hip_check(hipStreamSynchronize(plan->stream), "hipStreamSynchronize");
      if (rc) return rc;
      (void)hipFree(plan->rn64);
      (void)hipFree(plan->rn32);
      plan->rn64 = nullptr;
      plan->rn32 = nullptr;
      drop_precond(plan);
    }
    return CHEB_OK;
  }
  std::vector<double> h(cnt);
  int rc = hip_check(hipMemcpyAsync(h.data(), sigma_faces, cnt * sizeof(double), hipMemcpyDefault, plan->stream),
                     "hipMemcpyAsync(Robin coefficients)");
  if (!rc) rc = hip_check(hipStreamSynchronize(plan->stream), "hipStreamSynchronize");
  if (rc) return rc;
  double mean[6];
  for (int f = 0; f < 6; ++f) {
    const long long o = face_offset(f, n), m = face_offset(f + 1, n) - o;
    double s = 0.0;
    for (long long i = 0; i < m; ++i) {
      const double v = h[o + i];
      if (!std::isfinite(v) || (plan->g.bc[f] == CHEB_DIRICHLET && v != 0.0)) {
        set_error("per-node Robin coefficients must be finite, and 0 on Dirichlet faces");
        return CHEB_ERR_INVALID_ARG;
      }
      s += v;
    }
    mean[f] = m > 0 ? s / double(m) : 0.0;
  }
  // every pencil's end-value block with its own nodes' coefficients (as the
  // per-face check of cheb_plan_create)
  for (int a = 0; a < 3; ++a) {
    const AxisConst& c = plan->ax[a];
    const bool nlo = plan->g.bc[2 * a] == CHEB_NEUMANN, nhi = plan->g.bc[2 * a + 1] == CHEB_NEUMANN;
    if (!nlo && !nhi) continue;
    const double r00 = c.m00 + plan->g.robin[2 * a], rNN = c.mNN - plan->g.robin[2 * a + 1];
    const long long olo = face_offset(2 * a, n), ohi = face_offset(2 * a + 1, n);
    for (int p = 0; p < pencil_count(a, n); ++p) {
      const double m00 = c.m00 - h[olo + p], mNN = c.mNN + h[ohi + p];
      const double det = m00 * mNN - c.m0N * c.mN0;
      const double scale = std::fabs(m00 * mNN) + std::fabs(c.m0N * c.mN0);
      if ((nlo && !(std::fabs(m00) > 1e-12 * std::fabs(r00))) || (nhi && !(std::fabs(mNN) > 1e-12 * std::fabs(rNN))) ||
          (nlo && nhi && !(std::fabs(det) > 1e-12 * scale))) {
        set_error("per-node Robin coefficients make a boundary elimination block singular");
        return CHEB_ERR_INVALID_ARG;
      }
    }
  }
  // each pencil's end-block inverse, for the matrix-core pass (the FFT route
  // and the lifts solve the block from the coefficients themselves)
  h.resize(3 * cnt, 0.0);
  for (int a = 0; a < 3; ++a) {
    const AxisConst& c = plan->ax[a];
    const bool nlo = plan->g.bc[2 * a] == CHEB_NEUMANN, nhi = plan->g.bc[2 * a + 1] == CHEB_NEUMANN;
    const long long olo = face_offset(2 * a, n), ohi = face_offset(2 * a + 1, n);
    double* e = h.data() + robin_inv_offset(plan, a);
    for (int p = 0; p < pencil_count(a, n); ++p, e += 4) {
      const double m00 = c.m00 - h[olo + p], mNN = c.mNN + h[ohi + p];
      if (nlo && nhi) {
        const double det = m00 * mNN - c.m0N * c.mN0;
        e[0] = mNN / det;
        e[1] = -c.m0N / det;
        e[2] = -c.mN0 / det;
        e[3] = m00 / det;
      } else if (nlo) {
        e[0] = 1.0 / m00;
      } else if (nhi) {
        e[3] = 1.0 / mNN;
      }
    }
  }
  const size_t tot = 3 * cnt;
  std::vector<float> h32(tot);
  for (size_t i = 0; i < tot; ++i) h32[i] = float(h[i]);
  rc = CHEB_OK;
  if (!plan->rn64) {
    rc = hip_check(hipMalloc((void**)&plan->rn64, tot * sizeof(double)), "hipMalloc(Robin coefficients)");
    if (!rc) rc = hip_check(hipMalloc((void**)&plan->rn32, tot * sizeof(float)), "hipMalloc(Robin coefficients)");
    if (rc) {
      if (plan->rn64) (void)hipFree(plan->rn64);
      plan->rn64 = nullptr;
      plan->rn32 = nullptr;
      return rc;
    }
  }
  rc = hip_check(hipMemcpyAsync(plan->rn64, h.data(), tot * sizeof(double), hipMemcpyHostToDevice, plan->stream),
                 "hipMemcpyAsync(Robin coefficients)");
  if (!rc)
    rc = hip_check(hipMemcpyAsync(plan->rn32, h32.data(), tot * sizeof(float), hipMemcpyHostToDevice, plan->stream),
                   "hipMemcpyAsync(Robin coefficients)");
  if (!rc) rc = hip_check(hipStreamSynchronize(plan->stream), "hipStreamSynchronize");
  if (rc) {
    // the arrays may hold part of the new values: the plan drops its per-node part
    (void)hipFree(plan->rn64);
    (void)hipFree(plan->rn32);
    plan->rn64 = nullptr;
    plan->rn32 = nullptr;
    drop_precond(plan);
    return rc;
  }
  for (int f = 0; f < 6; ++f) plan->rn_mean[f] = mean[f];
  drop_precond(plan);
  return CHEB_OK;
}

int cheb_plan_set_route(cheb_plan* plan, int32_t route) {
  if (!plan) {
    set_error("null plan");
    return CHEB_ERR_INVALID_ARG;
  }
  if (route != CHEB_ROUTE_AUTO && route != CHEB_ROUTE_FFT && route != CHEB_ROUTE_MATRIX) {
    set_error("route must be CHEB_ROUTE_AUTO, CHEB_ROUTE_FFT or CHEB_ROUTE_MATRIX");
    return CHEB_ERR_INVALID_ARG;
  }
  plan->route = route;
  return CHEB_OK;
}

int cheb_plan_set_tile_shape(cheb_plan* plan, int32_t field_precision, int32_t shape) {
  if (!plan) {
    set_error("null plan");
    return CHEB_ERR_INVALID_ARG;
  }
  if (field_precision != CHEB_F64 && field_precision != CHEB_F32) {
    set_error("tile shape: field_precision must be CHEB_F64 or CHEB_F32");
    return CHEB_ERR_INVALID_ARG;
  }
  if (shape != 0 && shape != 1) {
    set_error("tile shape must be 0 (8-wave, LDS table) or 1 (4-wave, register fragments)");
    return CHEB_ERR_INVALID_ARG;
  }
  const int pi = field_precision == CHEB_F64 ? 0 : 1;
  for (int a = 0; a < 3; ++a) plan->dense_var[a][pi] = shape;
  return CHEB_OK;
}

int cheb_plan_destroy(cheb_plan* plan) {
  if (!plan) return CHEB_OK;
  if (plan->dconst64) (void)hipFree(plan->dconst64);
  if (plan->dconst32) (void)hipFree(plan->dconst32);
  if (plan->dd64) (void)hipFree(plan->dd64);
  if (plan->dd32) (void)hipFree(plan->dd32);
  if (plan->pair_buf) (void)hipFree(plan->pair_buf);
  if (plan->kev_ok) {
    (void)hipEventDestroy(plan->kev[0]);
    (void)hipEventDestroy(plan->kev[1]);
  }
  if (plan->hpinned) (void)hipHostFree(plan->hpinned);
  if (plan->pc64) (void)hipFree(plan->pc64);
  if (plan->pc32) (void)hipFree(plan->pc32);
  if (plan->rn64) (void)hipFree(plan->rn64);
  if (plan->rn32) (void)hipFree(plan->rn32);
  delete plan;
  return CHEB_OK;
}

int cheb_apply(cheb_plan* plan, const void* K, const void* u, void* y, uint32_t flags) {
  if (!plan || !K || !u || !y) {
    set_error("null argument");
    return CHEB_ERR_INVALID_ARG;
  }
  if (y == u || y == K) {
    set_error("output must not alias the input");
    return CHEB_ERR_INVALID_ARG;
  }
  int mode;
  if (flags == CHEB_APPLY_FULL) mode = 0;
  else if (flags == CHEB_APPLY_REDUCED) mode = 1;
  else if (flags == (CHEB_APPLY_REDUCED | CHEB_APPLY_TRANSPOSE)) mode = 2;
  else {
    set_error("flags must be FULL, REDUCED or REDUCED|TRANSPOSE");
    return CHEB_ERR_INVALID_ARG;
  }
  if (plan->prec == CHEB_F32)
    return apply_t<float>(plan, (const float*)K, (const float*)u, (float*)y, mode, plan->stream);
  return apply_t<double>(plan, (const double*)K, (const double*)u, (double*)y, mode, plan->stream);
}

int cheb_plan_autotune(cheb_plan* plan, int32_t field_precision, const void* K, const void* u, void* y,
                       double* report, int32_t report_len) {
  if (!plan || !K || !u || !y || y == u || y == K || (report_len > 0 && !report)) {
    set_error("invalid argument");
    return CHEB_ERR_INVALID_ARG;
  }
  if (field_precision == CHEB_F64 && plan->prec != CHEB_F32)
    return autotune_t<double>(plan, (const double*)K, (const double*)u, (double*)y, report, report_len);
  if (field_precision == CHEB_F32 && plan->prec != CHEB_F64)
    return autotune_t<float>(plan, (const float*)K, (const float*)u, (float*)y, report, report_len);
  set_error("field precision must match the plan (F64 plan: CHEB_F64; F32 plan: CHEB_F32; MIXED: either)");
  return CHEB_ERR_INVALID_ARG;
}

int cheb_derivative(cheb_plan* plan, const void* u, void* du, int32_t axis) {
  if (!plan || !u || !du || axis < 0 || axis > 2 || u == du) {
    set_error("invalid argument");
    return CHEB_ERR_INVALID_ARG;
  }
  if (plan->prec == CHEB_F32)
    return launch_axis_pass<float>(plan, axis, 3, 1, nullptr, (const float*)u, (float*)du, plan->stream);
  return launch_axis_pass<double>(plan, axis, 3, 1, nullptr, (const double*)u, (double*)du, plan->stream);
}

int cheb_flux_average(cheb_plan* plan, const void* K, const void* u, double out[3]) {
  if (!plan || !K || !u || !out) {
    set_error("null argument");
    return CHEB_ERR_INVALID_ARG;
  }
  if (plan->prec == CHEB_F32) {
    set_error("flux average needs an FP64 or MIXED plan");
    return CHEB_ERR_UNSUPPORTED;
  }
  const size_t fb = round_up(plan->npts * sizeof(double), 256);
  const size_t pb = round_up(8192 * sizeof(double), 256);
  if (!plan->ws || plan->ws_bytes < fb + pb) {
    set_error("flux average needs the workspace");
    return CHEB_ERR_WORKSPACE;
  }
  double* du = (double*)plan->ws;
  double* part = (double*)((char*)plan->ws + fb);
  double* res = part + 4096;
  const double vol = (plan->g.hi[0] - plan->g.lo[0]) * (plan->g.hi[1] - plan->g.lo[1]) *
                     (plan->g.hi[2] - plan->g.lo[2]);
  for (int b = 0; b < 3; ++b) {
    int rc = launch_axis_pass<double>(plan, b, 3, 1, nullptr, (const double*)u, du, plan->stream);
    if (rc) return rc;
    rc = cc_dot((const double*)K, du, dconst64(plan, 0, 2), dconst64(plan, 1, 2), dconst64(plan, 2, 2),
                plan->g.n, part, res + b, plan->stream);
    if (rc) return rc;
  }
  int rc = hip_check(hipMemcpyAsync(plan->hpinned, res, 3 * sizeof(double), hipMemcpyDeviceToHost, plan->stream),
                     "hipMemcpyAsync");
  if (rc) return rc;
  rc = hip_check(hipStreamSynchronize(plan->stream), "hipStreamSynchronize");
  if (rc) return rc;
  for (int b = 0; b < 3; ++b) out[b] = plan->hpinned[b] / vol;
  return CHEB_OK;
}

int cheb_apparent_conductivity(cheb_plan* plan, const void* K, const void* u, int32_t axis, double jump,
                               double out[3]) {
  if (!plan || !out || axis < 0 || axis > 2 || !(jump != 0.0) || !std::isfinite(jump)) {
    set_error("apparent conductivity: null argument, axis outside 0..2 or zero / non-finite jump");
    return CHEB_ERR_INVALID_ARG;
  }
  double fl[3];
  const int rc = cheb_flux_average(plan, K, u, fl);
  if (rc) return rc;
  // Section 3.3: K_app[b][axis] = <K du/dx_b> / G with the imposed mean gradient G
  const double G = jump / (plan->g.hi[axis] - plan->g.lo[axis]);
  for (int b = 0; b < 3; ++b) out[b] = fl[b] / G;
  return CHEB_OK;
}

}  // extern "C"
