// Solvers behind the C ABI: LGMRES on the reduced system (Algorithm 2), FP32
// LGMRES inside FP64 iterative refinement, the adjoint solve and gradient, and
// the Picard loop.  All arithmetic runs in device kernels, the (m+k+1) x (m+k)
// Hessenberg matrix, its Givens rotations and the convergence test of each
// Arnoldi step included (krylov.hip); the host enqueues the steps and reads
// one small status record per step, one step behind the GPU.
//
// LGMRES (Baker, Jessup & Manteuffel, SIAM J. Matrix Anal. Appl. 26(4), 2005):
// each restart cycle builds an Arnoldi basis from the residual and then
// continues the Arnoldi process with the k most recent corrections
// z_i = x_i - x_{i-1} as extra search directions; the update is the
// least-squares minimiser over that augmented space.  Orthogonalisation is
// classical Gram-Schmidt in one pass: the multi-dot returns <v_i, w> and <w, w>
// together; ||w - V h||^2 = ||w||^2 - ||h||^2, and a second pass runs when
// that difference signals severe cancellation, ||w_new|| < ||w|| / 10 (the
// criterion of Daniel, Gragg, Kaufman and Stewart with eta = 0.1; at 1/sqrt(2)
// the second pass ran on nearly every step here, to no effect on convergence).
#include <chrono>
#include <cmath>
#include <vector>

#include "internal.h"

namespace cheb {

namespace {

struct Carver {
  char* base;
  size_t off;
  template <typename T>
  T* take(size_t count) {
    T* p = base ? (T*)(base + off) : nullptr;
    off += round_up(count * sizeof(T), 256);
    return p;
  }
};

struct SolveParams {
  double rtol, atol;
  int maxiter, m, k;
  double ir_rtol;
  int ir_max;
  bool warm;
  bool precond;
  double* hist;
  int hist_len;
};

SolveParams params_from(const cheb_solve_opts* o) {
  SolveParams s;
  s.rtol = (o && o->rtol > 0) ? o->rtol : 1e-10;
  s.atol = (o && o->atol > 0) ? o->atol : 0.0;
  s.maxiter = (o && o->maxiter > 0) ? o->maxiter : 10000;
  s.m = (o && o->inner_m > 0) ? o->inner_m : 30;
  s.k = !o || o->outer_k == 0 ? 3 : (o->outer_k < 0 ? 0 : o->outer_k);
  s.ir_rtol = (o && o->ir_inner_rtol > 0) ? o->ir_inner_rtol : 1e-3;
  s.ir_max = (o && o->ir_max_outer > 0) ? o->ir_max_outer : 50;
  s.warm = o && (o->flags & 1);
  s.precond = o && (o->flags & 2);
  s.hist = o ? o->history : nullptr;
  s.hist_len = o ? o->history_len : 0;
  return s;
}

template <typename T>
struct KrylovWS {
  T* V = nullptr;   // m + k + 1 basis vectors
  T* Z = nullptr;   // k augmentation vectors (corrections of earlier cycles, solution space)
  T* w = nullptr;   // work vectors: A d_j of even and odd steps (a step enqueued past a pause
  T* w2 = nullptr;  // of the cycle must not overwrite the paused step's vector)
  T* D = nullptr;   // m preconditioned directions M^{-1} v_j (flexible form; only with a preconditioner)
  T* pa = nullptr;  // packed-interior scratch of the preconditioner
  T* pb = nullptr;
  size_t ld = 0;    // elements between vectors
  int m = 0, k = 0;
};

struct Scratch {
  double* partials = nullptr;
  double* dots = nullptr;   // device, 2 x 80
  double* coef = nullptr;   // device, 80
  int* flag = nullptr;
  ArnoldiState* ast = nullptr;  // device state of the restart cycle
};

template <typename T>
void carve_krylov(Carver& c, const cheb_plan* p, int m, int k, bool prec, KrylovWS<T>& kw) {
  const size_t npts = p->npts;
  kw.ld = round_up(npts * sizeof(T), 256) / sizeof(T);
  kw.m = m;
  kw.k = k;
  kw.V = c.take<T>(kw.ld * (m + k + 1));
  kw.Z = c.take<T>(kw.ld * (k > 0 ? k : 1));
  kw.w = c.take<T>(kw.ld);
  kw.w2 = c.take<T>(kw.ld);
  if (prec) {
    const size_t inner = (size_t)(p->g.n[0] - 2) * (p->g.n[1] - 2) * (p->g.n[2] - 2);
    kw.D = c.take<T>(kw.ld * m);
    kw.pa = c.take<T>(inner);
    kw.pb = c.take<T>(inner);
  }
}

void carve_scratch(Carver& c, size_t npts, int maxv, Scratch& s) {
  s.partials = c.take<double>(multidot_partials_len(npts, maxv));
  s.dots = c.take<double>(160);
  s.coef = c.take<double>(80);
  s.flag = c.take<int>(64);
  s.ast = c.take<ArnoldiState>(1);
}

struct Stats {
  int matvecs = 0;
  int restarts = 0;
  int hist_used = 0;
};

// read back `cnt` doubles from device `src` into the plan's pinned buffer
int readback(cheb_plan* p, const double* src, int cnt, double* dst, int slot = 0) {
  double* hp = p->hpinned + slot * 256;
  int rc = hip_check(hipMemcpyAsync(hp, src, cnt * sizeof(double), hipMemcpyDeviceToHost, p->stream),
                     "hipMemcpyAsync(D2H)");
  if (rc) return rc;
  rc = hip_check(hipStreamSynchronize(p->stream), "hipStreamSynchronize");
  if (rc) return rc;
  for (int i = 0; i < cnt; ++i) dst[i] = hp[i];
  return CHEB_OK;
}

template <typename T>
int vnorm(cheb_plan* p, const T* v, Scratch& s, double* out) {
  int rc = multidot<T>(nullptr, 0, 0, v, p->npts, s.partials, s.dots, p->stream);
  if (rc) return rc;
  double ww;
  rc = readback(p, s.dots, 1, &ww);
  if (rc) return rc;
  *out = std::sqrt(ww > 0 ? ww : 0.0);
  return CHEB_OK;
}

// completion events of the last two Arnoldi steps (created once per plan)
int ensure_events(cheb_plan* p) {
  if (p->kev_ok) return CHEB_OK;
  int rc = hip_check(hipEventCreateWithFlags(&p->kev[0], hipEventDisableTiming), "hipEventCreate");
  if (rc) return rc;
  rc = hip_check(hipEventCreateWithFlags(&p->kev[1], hipEventDisableTiming), "hipEventCreate");
  if (rc) {
    (void)hipEventDestroy(p->kev[0]);
    return rc;
  }
  p->kev_ok = 1;
  return CHEB_OK;
}

// LGMRES on  A x = b  with absolute tolerance tol_abs on ||b - A x||.
// Returns CHEB_OK when converged, CHEB_NOT_CONVERGED when maxmv was reached.
// stall > 0: stop with CHEB_STAGNATED when a restart cycle reduces the true
// residual by less than that factor (used by the FP32 inner solves, whose
// attainable accuracy is bounded by the FP32 operator).
//
// With a preconditioner the cycle is the flexible form of right
// preconditioning: the directions d_j = M^{-1} v_j are kept, and the update is
// sum_j y_j d_j, so the minimised residual is that of the directions actually
// applied (the preconditioner need not be the same linear map at every step;
// with one that is, this is ordinary right preconditioning).  Augmentation
// vectors are earlier corrections x_i - x_{i-1}, used as directions directly.
//
// Every Arnoldi step is enqueued without a host wait: the Hessenberg column,
// the rotations and the convergence predicate run on the device
// (krylov.hip), the re-orthogonalisation kernels run or not by a device flag,
// and the host reads the step's status record one step later, so at most one
// step is enqueued past the end of a cycle (its column kernel then does
// nothing).
struct NoPrec {
  template <typename T>
  int operator()(const T*, T*) const { return CHEB_OK; }
};

template <typename T, typename ApplyFn, typename PrecFn = NoPrec>
int lgmres(cheb_plan* p, ApplyFn&& A, const T* b, T* x, bool x_zero, double tol_abs, int maxmv,
           KrylovWS<T>& kw, Scratch& sc, Stats& st, double* resid_out, double bnorm, double* hist,
           int hist_len, double stall = 0.0, bool use_prec = false, PrecFn&& Mi = PrecFn(),
           std::vector<int>* zkeep = nullptr) {
  const size_t npts = p->npts;
  hipStream_t s = p->stream;
  const int m = kw.m, kmax = kw.k;
  const size_t ld = kw.ld;
  // augmentation vectors, most recent first; with zkeep they persist across
  // calls on the same operator (the corrections of earlier solves stay search
  // directions of the next one)
  std::vector<int> zlocal;
  std::vector<int>& zslot = zkeep ? *zkeep : zlocal;
  T* w = kw.w;
  ArnoldiState* ast = sc.ast;
  double* dots2 = sc.dots + 80;
  ArnoldiHead* ring = (ArnoldiHead*)(p->hpinned + 4 * 256);  // two pinned status slots
  int rc = ensure_events(p);
  if (!rc) rc = arnoldi_init(ast, tol_abs, stall, s);
  if (rc) return rc;
  bool first = true;
  for (;;) {
    // true residual r = b - A x into V_0, then v_0 = r / ||r|| (device scale)
    T* v0 = kw.V;
    if (first && x_zero) {
      rc = copy_scale<T>(v0, b, 1.0, npts, s);
    } else {
      rc = A(x, v0);
      if (!rc) rc = axpby<T>(v0, b, 1.0, -1.0, npts, s);
      st.matvecs++;
    }
    first = false;
    if (!rc) rc = multidot<T>(nullptr, 0, 0, v0, npts, sc.partials, sc.dots, s);
    if (!rc) rc = arnoldi_begin(ast, sc.dots, s);
    if (!rc) rc = scale_by<T>(v0, &ast->inv_beta, npts, s);
    if (rc) return rc;
    int jmax = m + (int)zslot.size();
    if (jmax > maxmv - st.matvecs) jmax = maxmv - st.matvecs;
    // one Arnoldi step: direction, operator, Gram-Schmidt pass 0 and column j
    // on the device, v_{j+1} unless the column ended or paused the cycle
    auto step = [&](int j) -> int {
      // the operator and preconditioner kernels of the step do nothing once
      // the cycle has ended (or paused) on the device
      struct Gate {
        cheb_plan* p;
        ~Gate() { p->gate = nullptr; }
      } gate{p};
      p->gate = &ast->active;
      const T* dir;
      if (j >= m) {
        dir = kw.Z + (size_t)zslot[j - m] * ld;
      } else if (use_prec) {
        T* dj = kw.D + (size_t)j * ld;
        int r = Mi(kw.V + (size_t)j * ld, dj);
        if (r) return r;
        dir = dj;
      } else {
        dir = kw.V + (size_t)j * ld;
      }
      T* wj = (j & 1) ? kw.w2 : w;
      int r = A(dir, wj);
      p->gate = nullptr;
      // the column kernel also writes the step's head to its pinned ring slot
      if (!r) r = gram_schmidt<T>(kw.V, ld, j, wj, npts, nullptr, sc.partials, sc.dots, ast, 0, s, &ring[j & 1]);
      if (!r)
        r = update_scale<T>(kw.V, ld, j + 1, sc.dots, wj, kw.V + (size_t)(j + 1) * ld, 1.0, npts, s, &ast->inv_hn,
                            &ast->direct);
      return r;
    };
    auto fetch_now = [&](ArnoldiHead* out) -> int {
      int r = hip_check(hipMemcpyAsync(&ring[0], ast, sizeof(ArnoldiHead), hipMemcpyDeviceToHost, s),
                        "hipMemcpyAsync(D2H)");
      if (!r) r = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
      if (!r) *out = ring[0];
      return r;
    };
    ArnoldiHead h;
    int jnext = 0;
    bool any = false;
    for (;;) {
      // enqueue steps jnext.. with the status of each read one step later
      int last = -1;
      for (int j = jnext; j < jmax; ++j) {
        rc = step(j);
        if (!rc) rc = hip_check(hipEventRecord(p->kev[j & 1], s), "hipEventRecord");
        if (rc) return rc;
        last = j;
        any = true;
        if (j > jnext) {
          rc = hip_check(hipEventSynchronize(p->kev[(j - 1) & 1]), "hipEventSynchronize");
          if (rc) return rc;
          if (!ring[(j - 1) & 1].active) break;
        }
      }
      if (last >= 0) {
        rc = hip_check(hipEventSynchronize(p->kev[last & 1]), "hipEventSynchronize");
        if (rc) return rc;
        h = ring[last & 1];
      } else {
        rc = fetch_now(&h);
        if (rc) return rc;
      }
      if (!(h.reorth && h.beta > tol_abs && !h.stagnated)) break;
      // paused at column jc by cancellation: the second Gram-Schmidt pass for
      // it (any step enqueued after it ran on a stale vector and is redone)
      const int jc = h.jend;
      T* wc = (jc & 1) ? kw.w2 : w;
      rc = gram_schmidt<T>(kw.V, ld, jc, wc, npts, sc.dots, sc.partials, dots2, ast, 1, s);
      if (!rc)
        rc = update_scale<T>(kw.V, ld, jc + 1, dots2, wc, kw.V + (size_t)(jc + 1) * ld, 1.0, npts, s,
                             &ast->inv_hn, &ast->direct);
      if (!rc) rc = fetch_now(&h);
      if (rc) return rc;
      jnext = jc + 1;
      if (!h.active || jnext >= jmax) break;
    }
    const int enq = any ? 1 : 0;
    const double beta = h.beta;
    if (hist && st.hist_used < hist_len) hist[st.hist_used++] = bnorm > 0 ? beta / bnorm : beta;
    *resid_out = beta;
    if (!(beta > tol_abs)) return std::isfinite(beta) ? CHEB_OK : CHEB_NOT_CONVERGED;
    if (h.stagnated) return CHEB_STAGNATED;
    if (enq == 0) return CHEB_NOT_CONVERGED;
    const int jend = h.jend;
    st.matvecs += jend;
    // dx = sum_{j<m} y_j d_j + sum_{j>=m} y_j z_{j-m}  (into w), x += dx
    rc = arnoldi_solve(ast, s);
    const int nv = jend < m ? jend : m;
    if (!rc) rc = lincomb<T>(use_prec ? kw.D : kw.V, ld, nv, ast->y, w, 0, npts, s);
    for (int i = m; i < jend && !rc; ++i)
      rc = lincomb<T>(kw.Z + (size_t)zslot[i - m] * ld, ld, 1, ast->y + i, w, 1, npts, s);
    if (!rc) rc = axpby<T>(x, w, 1.0, 1.0, npts, s);
    if (!rc && kmax > 0) {
      // store the correction as the newest augmentation vector
      int slot;
      if ((int)zslot.size() < kmax) {
        slot = (int)zslot.size();
      } else {
        slot = zslot.back();
        zslot.pop_back();
      }
      rc = copy_scale<T>(kw.Z + (size_t)slot * ld, w, 1.0, npts, s);
      zslot.insert(zslot.begin(), slot);
    }
    if (rc) return rc;
    st.restarts++;
  }
}

size_t field_bytes(size_t npts, size_t elem) { return round_up(npts * elem, 256); }

// workspace carving for each entry point; base == nullptr gives the size
struct SolveWS64 {
  double *bt, *x, *r, *t1, *t2, *t3;
  KrylovWS<double> kw;
  Scratch sc;
};
struct SolveWS32 {
  float *bt, *x, *K, *f, *g;
  KrylovWS<float> kw;
  Scratch sc;
};
struct MixedWS {
  double *bt, *x, *r, *t1;
  float *K32, *b32, *d32;
  KrylovWS<float> kw;
  Scratch sc;
};

size_t carve64(cheb_plan* p, const SolveParams& sp, char* base, SolveWS64& w) {
  Carver c{base, 0};
  w.bt = c.take<double>(p->npts);
  w.x = c.take<double>(p->npts);
  w.r = c.take<double>(p->npts);
  w.t1 = c.take<double>(p->npts);
  w.t2 = c.take<double>(p->npts);
  w.t3 = c.take<double>(p->npts);
  carve_krylov<double>(c, p, sp.m, sp.k, sp.precond, w.kw);
  carve_scratch(c, p->npts, sp.m + sp.k + 2, w.sc);
  return c.off;
}

size_t carve32(cheb_plan* p, const SolveParams& sp, char* base, SolveWS32& w) {
  Carver c{base, 0};
  w.bt = c.take<float>(p->npts);
  w.x = c.take<float>(p->npts);
  w.K = nullptr;
  w.f = nullptr;
  w.g = nullptr;
  carve_krylov<float>(c, p, sp.m, sp.k, sp.precond, w.kw);
  carve_scratch(c, p->npts, sp.m + sp.k + 2, w.sc);
  return c.off;
}

size_t carve_mixed(cheb_plan* p, const SolveParams& sp, char* base, MixedWS& w) {
  Carver c{base, 0};
  w.bt = c.take<double>(p->npts);
  w.x = c.take<double>(p->npts);
  w.r = c.take<double>(p->npts);
  w.t1 = c.take<double>(p->npts);
  w.K32 = c.take<float>(p->npts);
  w.b32 = c.take<float>(p->npts);
  w.d32 = c.take<float>(p->npts);
  carve_krylov<float>(c, p, sp.m, sp.k, sp.precond, w.kw);
  carve_scratch(c, p->npts, sp.m + sp.k + 2, w.sc);
  return c.off;
}

size_t solve_need(cheb_plan* p, const SolveParams& sp) {
  SolveWS64 w64;
  SolveWS32 w32;
  MixedWS wm;
  if (p->prec == CHEB_F32) return carve32(p, sp, nullptr, w32);
  size_t need = carve64(p, sp, nullptr, w64);
  if (p->prec == CHEB_MIXED) {
    const size_t mb = carve_mixed(p, sp, nullptr, wm);
    if (mb > need) need = mb;
  }
  return need;
}

int check_K(cheb_plan* p, const void* K, Scratch& sc) {
  int rc = hip_check(hipMemsetAsync(sc.flag, 0, sizeof(int), p->stream), "hipMemsetAsync");
  if (rc) return rc;
  if (p->prec == CHEB_F32) rc = check_positive_finite_f32((const float*)K, p->npts, sc.flag, p->stream);
  else rc = check_positive_finite((const double*)K, p->npts, sc.flag, p->stream);
  if (rc) return rc;
  int* hf = (int*)(p->hpinned + 3 * 256);
  rc = hip_check(hipMemcpyAsync(hf, sc.flag, sizeof(int), hipMemcpyDeviceToHost, p->stream), "hipMemcpyAsync");
  if (rc) return rc;
  rc = hip_check(hipStreamSynchronize(p->stream), "hipStreamSynchronize");
  if (rc) return rc;
  if (*hf) {
    set_error("conductivity must be finite and positive at every node");
    return CHEB_ERR_BAD_INPUT;
  }
  return CHEB_OK;
}

// reduced right-hand side bt = f_k - A_kr H g (interior), 0 on the boundary
template <typename T>
int reduced_rhs(cheb_plan* p, const T* K, const T* f, const T* g, T* bt, T* tmp) {
  int rc = fill<T>(tmp, 0.0, p->npts, p->stream);
  if (!rc) rc = lift_full<T>(p, tmp, g, p->stream);
  if (!rc) rc = apply_t<T>(p, K, tmp, bt, 0, p->stream);
  if (!rc) rc = rhs_reduced<T>(bt, f, p->g.n, p->stream);
  return rc;
}

// FP64 (or FP32) plain LGMRES solve of the reduced system; x holds interior values.
// mean of K (scale of the preconditioner's constant-coefficient operator)
template <typename T>
int mean_K(cheb_plan* p, const T* K, Scratch& sc, double* kc) {
  int rc = vsum<T>(K, p->npts, sc.partials, sc.dots, p->stream);
  if (rc) return rc;
  double sum;
  rc = readback(p, sc.dots, 1, &sum);
  if (rc) return rc;
  *kc = sum / double(p->npts);
  return CHEB_OK;
}

template <typename T>
int solve_plain(cheb_plan* p, const T* K, const T* bt, T* x, T* r, KrylovWS<T>& kw, Scratch& sc,
                const SolveParams& sp, int mode, Stats& st, double* relres, int* status) {
  double bnorm;
  int rc = vnorm<T>(p, bt, sc, &bnorm);
  if (rc) return rc;
  const double tol = std::fmax(sp.rtol * bnorm, sp.atol);
  auto A = [&](const T* in, T* out) { return apply_t<T>(p, K, in, out, mode, p->stream); };
  double res = 0;
  if (bnorm == 0.0) {
    rc = fill<T>(x, 0.0, p->npts, p->stream);
    *relres = 0.0;
    *status = CHEB_OK;
    return rc;
  }
  double kc = 1.0;
  if (sp.precond) {
    rc = precond_setup(p);
    if (!rc) rc = mean_K<T>(p, K, sc, &kc);
    if (rc) return rc;
  }
  auto Mi = [&](const T* in, T* out) {
    return precond_apply<T>(p, in, out, kw.pa, kw.pb, kc, mode == 2, p->stream);
  };
  const int r2 = lgmres<T>(p, A, bt, x, !sp.warm, tol, sp.maxiter, kw, sc, st, &res, bnorm, sp.hist,
                           sp.hist_len, 0.0, sp.precond, Mi);
  if (r2 < 0) return r2;
  *status = r2;
  // final true residual
  rc = A(x, r);
  if (!rc) rc = axpby<T>(r, bt, 1.0, -1.0, p->npts, p->stream);
  if (rc) return rc;
  double rn;
  rc = vnorm<T>(p, r, sc, &rn);
  if (rc) return rc;
  *relres = rn / bnorm;
  return CHEB_OK;
}


// Newton iteration for k(x, T) = K0(x) / (1 + alpha T) (Section 3.4).  Fields of
// the caller's work array, each padded to 256 bytes: k(T), c_a = k'(T) D_a T for
// a = 0, 1, 2, the lifted direction (also k'(T) while linearising) and a
// 256-byte flag slot.
constexpr int kNewtonFields = 5;

struct NewtonWS {
  double *k, *c[3], *V;
  int* flag;
};

NewtonWS newton_ws(const cheb_plan* p, void* work) {
  Carver c{(char*)work, 0};
  NewtonWS w;
  w.k = c.take<double>(p->npts);
  for (int a = 0; a < 3; ++a) w.c[a] = c.take<double>(p->npts);
  w.V = c.take<double>(p->npts);
  w.flag = c.take<int>(64);
  return w;
}

// k and c_a at the state T (full nodal array); fails when 1 + alpha T <= 0
// somewhere, where the law has no positive conductivity.
int newton_linearise(cheb_plan* p, const double* K0, double alpha, const double* T, NewtonWS& w) {
  int rc = newton_coeff(w.k, w.V, K0, T, alpha, p->npts, p->stream);
  for (int a = 0; a < 3 && !rc; ++a) {
    rc = launch_axis_pass<double>(p, a, 3, 1, nullptr, T, w.c[a], p->stream);
    if (!rc) rc = vmul(w.c[a], w.c[a], w.V, p->npts, p->stream);
  }
  if (!rc) rc = hip_check(hipMemsetAsync(w.flag, 0, sizeof(int), p->stream), "hipMemsetAsync");
  if (!rc) rc = check_positive_finite(w.k, p->npts, w.flag, p->stream);
  if (rc) return rc;
  int* hf = (int*)(p->hpinned + 3 * 256);
  rc = hip_check(hipMemcpyAsync(hf, w.flag, sizeof(int), hipMemcpyDeviceToHost, p->stream), "hipMemcpyAsync");
  if (!rc) rc = hip_check(hipStreamSynchronize(p->stream), "hipStreamSynchronize");
  if (rc) return rc;
  if (*hf) {
    set_error("k(T) = K0 / (1 + alpha T) must be finite and positive at every node (check K0 and 1 + alpha T)");
    return CHEB_ERR_BAD_INPUT;
  }
  return CHEB_OK;
}

// y = J(T) v on interior rows (boundary rows 0): the reduced operator with
// coefficient k(T), plus sum_a D_a (c_a V) with V the homogeneous lift of v.
// On the matrix-core route the c_a terms join the reduced apply's flux
// epilogues; otherwise each axis' term is one accumulating derivative pass
// that lifts v's interior values in the pencil (as the reduced operator does)
// and multiplies by c_a.
int newton_jv(cheb_plan* p, NewtonWS& w, const double* v, double* y) {
  hipStream_t s = p->stream;
  // matrix-core route with the x and y passes in one launch: the c_a terms
  // ride in the reduced apply's flux epilogues (two launches in all)
  const double* c[3] = {w.c[0], w.c[1], w.c[2]};
  const int r = launch_dense_jac<double>(p, w.k, c, v, y, s);
  if (r != CHEB_ERR_UNSUPPORTED) return r;
  int rc = apply_t<double>(p, w.k, v, y, 1, s);
  for (int a = 0; a < 3 && !rc; ++a) rc = launch_axis_pass<double>(p, a, 5, 0, w.c[a], v, y, s);
  return rc;
}

// out = -R(T) = f - sum_a D_a (k D_a T) on interior rows, 0 on boundary rows
int newton_neg_residual(cheb_plan* p, NewtonWS& w, const double* T, const double* f, double* out) {
  int rc = apply_t<double>(p, w.k, T, out, 0, p->stream);
  if (!rc) rc = rhs_reduced<double>(out, f, p->g.n, p->stream);
  return rc;
}

int newton_check_plan(const cheb_plan* p) {
  if (p->prec == CHEB_F32) {
    set_error("Newton needs an FP64 or MIXED plan");
    return CHEB_ERR_UNSUPPORTED;
  }
  return CHEB_OK;
}

}  // namespace
}  // namespace cheb

using namespace cheb;

extern "C" {

int cheb_plan_workspace_bytes(const cheb_plan* plan, const cheb_solve_opts* opts, size_t* bytes) {
  if (!plan || !bytes) {
    set_error("null argument");
    return CHEB_ERR_INVALID_ARG;
  }
  // solver layout, then two FP64 fields used by the Picard loop, the
  // prolongation and the flux averages
  *bytes = solve_need(const_cast<cheb_plan*>(plan), params_from(opts)) +
           2 * field_bytes(plan->npts, sizeof(double));
  return CHEB_OK;
}

int cheb_solve(cheb_plan* plan, const void* K, const void* f, const void* g_faces, void* u_inout,
               const cheb_solve_opts* opts, cheb_solve_info* info) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!plan || !K || !f || !g_faces || !u_inout) {
    set_error("null argument");
    return CHEB_ERR_INVALID_ARG;
  }
  cheb_plan* p = plan;
  const SolveParams sp = params_from(opts);
  if (sp.m < 1 || sp.m > 64 || sp.k < 0 || sp.k > 6) {
    set_error("inner_m must be in [1, 64] and outer_k in [0, 6]");
    return CHEB_ERR_INVALID_ARG;
  }
  size_t need = 0;
  if (cheb_plan_workspace_bytes(plan, opts, &need)) return CHEB_ERR_INVALID_ARG;
  if (!p->ws || p->ws_bytes < need) {
    set_error("workspace missing or too small (see cheb_plan_workspace_bytes)");
    return CHEB_ERR_WORKSPACE;
  }
  cheb_solve_info inf{};
  Stats st;
  int rc = 0;
  int status = CHEB_OK;
  double relres = 0;
  if (p->prec == CHEB_F64) {
    SolveWS64 w;
    carve64(p, sp, (char*)p->ws, w);
    rc = check_K(p, K, w.sc);
    if (rc) return rc;
    const double* Kd = (const double*)K;
    rc = reduced_rhs<double>(p, Kd, (const double*)f, (const double*)g_faces, w.bt, w.t1);
    if (!rc) {
      if (sp.warm) {
        rc = copy_scale<double>(w.x, (const double*)u_inout, 1.0, p->npts, p->stream);
        if (!rc) rc = mask_interior<double>(w.x, p->g.n, p->stream);
      } else {
        rc = fill<double>(w.x, 0.0, p->npts, p->stream);
      }
    }
    if (!rc) rc = solve_plain<double>(p, Kd, w.bt, w.x, w.r, w.kw, w.sc, sp, 1, st, &relres, &status);
    if (!rc) rc = copy_scale<double>((double*)u_inout, w.x, 1.0, p->npts, p->stream);
    if (!rc) rc = lift_full<double>(p, (double*)u_inout, (const double*)g_faces, p->stream);
  } else if (p->prec == CHEB_F32) {
    SolveWS32 w;
    carve32(p, sp, (char*)p->ws, w);
    rc = check_K(p, K, w.sc);
    if (rc) return rc;
    const float* Kf = (const float*)K;
    // the first Krylov vector doubles as scratch for the lift of the face data
    rc = reduced_rhs<float>(p, Kf, (const float*)f, (const float*)g_faces, w.bt, w.kw.w);
    if (!rc) {
      if (sp.warm) {
        rc = copy_scale<float>(w.x, (const float*)u_inout, 1.0, p->npts, p->stream);
        if (!rc) rc = mask_interior<float>(w.x, p->g.n, p->stream);
      } else {
        rc = fill<float>(w.x, 0.0, p->npts, p->stream);
      }
    }
    if (!rc) rc = solve_plain<float>(p, Kf, w.bt, w.x, w.kw.Z, w.kw, w.sc, sp, 1, st, &relres, &status);
    if (!rc) rc = copy_scale<float>((float*)u_inout, w.x, 1.0, p->npts, p->stream);
    if (!rc) rc = lift_full<float>(p, (float*)u_inout, (const float*)g_faces, p->stream);
  } else {
    // MIXED: FP64 iterative refinement around FP32 LGMRES
    MixedWS w;
    carve_mixed(p, sp, (char*)p->ws, w);
    rc = check_K(p, K, w.sc);
    if (rc) return rc;
    const double* Kd = (const double*)K;
    rc = reduced_rhs<double>(p, Kd, (const double*)f, (const double*)g_faces, w.bt, w.t1);
    if (!rc) rc = cast_f64_f32(w.K32, Kd, 1.0, p->npts, p->stream);
    if (!rc) {
      if (sp.warm) {
        rc = copy_scale<double>(w.x, (const double*)u_inout, 1.0, p->npts, p->stream);
        if (!rc) rc = mask_interior<double>(w.x, p->g.n, p->stream);
      } else {
        rc = fill<double>(w.x, 0.0, p->npts, p->stream);
      }
    }
    double bnorm = 0;
    if (!rc) rc = vnorm<double>(p, w.bt, w.sc, &bnorm);
    const double tol = std::fmax(sp.rtol * bnorm, sp.atol);
    auto A64 = [&](const double* in, double* out) { return apply_t<double>(p, Kd, in, out, 1, p->stream); };
    auto A32 = [&](const float* in, float* out) { return apply_t<float>(p, w.K32, in, out, 1, p->stream); };
    double kc = 1.0;
    if (!rc && sp.precond) {
      rc = precond_setup(p);
      if (!rc) rc = mean_K<double>(p, Kd, w.sc, &kc);
    }
    auto M32 = [&](const float* in, float* out) {
      return precond_apply<float>(p, in, out, w.kw.pa, w.kw.pb, kc, false, p->stream);
    };
    double prev = HUGE_VAL;
    int slow = 0;
    status = CHEB_NOT_CONVERGED;
    int f32mv = 0;
    std::vector<int> zkeep;  // the inner solves share their augmentation vectors
    for (int it = 0; !rc; ++it) {
      rc = A64(w.x, w.r);
      if (!rc) rc = axpby<double>(w.r, w.bt, 1.0, -1.0, p->npts, p->stream);
      if (rc) break;
      st.matvecs++;
      double rho;
      rc = vnorm<double>(p, w.r, w.sc, &rho);
      if (rc) break;
      relres = bnorm > 0 ? rho / bnorm : 0.0;
      if (sp.hist && st.hist_used < sp.hist_len) sp.hist[st.hist_used++] = relres;
      if (!(rho > tol)) {
        status = CHEB_OK;
        break;
      }
      if (it >= sp.ir_max || st.matvecs >= sp.maxiter) break;
      if (rho > 0.5 * prev) {
        if (++slow >= 3) {
          status = CHEB_STAGNATED;
          break;
        }
      } else {
        slow = 0;
      }
      prev = rho;
      inf.ir_steps++;
      rc = cast_f64_f32(w.b32, w.r, 1.0 / rho, p->npts, p->stream);
      if (!rc) rc = fill<float>(w.d32, 0.0, p->npts, p->stream);
      if (rc) break;
      Stats si;
      double res32 = 0;
      int budget = sp.maxiter - st.matvecs;
      const int cap = 40 * (sp.m + sp.k + 1);
      if (budget > cap) budget = cap;
      // the inner solve targets the reduction still needed (with a margin),
      // but not below ir_inner_rtol: a deep first solve, a short last one
      const double itol = std::fmax(sp.ir_rtol, 0.3 * tol / rho);
      const int r2 = lgmres<float>(p, A32, w.b32, w.d32, true, itol, budget > 1 ? budget : 1, w.kw,
                                   w.sc, si, &res32, 1.0, nullptr, 0, 0.9, sp.precond, M32, &zkeep);
      if (r2 < 0) {
        rc = r2;
        break;
      }
      st.matvecs += si.matvecs;
      f32mv += si.matvecs;
      st.restarts += si.restarts;
      rc = add_f32_to_f64(w.x, w.d32, rho, p->npts, p->stream);
    }
    inf.matvecs_f32 = f32mv;
    if (!rc) rc = copy_scale<double>((double*)u_inout, w.x, 1.0, p->npts, p->stream);
    if (!rc) rc = lift_full<double>(p, (double*)u_inout, (const double*)g_faces, p->stream);
  }
  if (!rc) rc = hip_check(hipStreamSynchronize(p->stream), "hipStreamSynchronize");
  if (rc) return rc;
  inf.status = status;
  inf.matvecs = st.matvecs;
  inf.restarts = st.restarts;
  inf.history_used = st.hist_used;
  inf.relres_final = relres;
  inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = inf;
  return status;
}

int cheb_adjoint(cheb_plan* plan, const void* K, const void* u, const void* dLdu, void* lambda, void* dLdlogK,
                 const cheb_solve_opts* opts, cheb_solve_info* info) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!plan || !K || !u || !dLdu || !lambda || !dLdlogK) {
    set_error("null argument");
    return CHEB_ERR_INVALID_ARG;
  }
  if (plan->prec == CHEB_F32) {
    set_error("the adjoint needs an FP64 or MIXED plan");
    return CHEB_ERR_UNSUPPORTED;
  }
  cheb_plan* p = plan;
  SolveParams sp = params_from(opts);
  if (sp.m < 1 || sp.m > 64 || sp.k < 0 || sp.k > 6) {
    set_error("inner_m must be in [1, 64] and outer_k in [0, 6]");
    return CHEB_ERR_INVALID_ARG;
  }
  sp.warm = false;
  SolveWS64 w;
  const size_t need = carve64(p, sp, nullptr, w);
  if (!p->ws || p->ws_bytes < need) {
    set_error("workspace missing or too small (see cheb_plan_workspace_bytes)");
    return CHEB_ERR_WORKSPACE;
  }
  carve64(p, sp, (char*)p->ws, w);
  int rc = check_K(p, K, w.sc);
  if (rc) return rc;
  const double* Kd = (const double*)K;
  // right-hand side r_k + G^T r_r
  rc = copy_scale<double>(w.bt, (const double*)dLdu, 1.0, p->npts, p->stream);
  if (!rc) rc = lift_transpose<double>(p, w.bt, p->stream);
  if (!rc) rc = fill<double>(w.x, 0.0, p->npts, p->stream);
  Stats st;
  double relres = 0;
  int status = CHEB_OK;
  if (!rc) rc = solve_plain<double>(p, Kd, w.bt, w.x, w.r, w.kw, w.sc, sp, 2, st, &relres, &status);
  if (!rc) rc = copy_scale<double>((double*)lambda, w.x, 1.0, p->npts, p->stream);
  // gradient  -K sum_a (D_a u)(D_a^T lambda~)
  for (int a = 0; a < 3 && !rc; ++a) {
    rc = launch_axis_pass<double>(p, a, 3, 1, nullptr, (const double*)u, w.t1, p->stream);
    if (!rc) rc = launch_axis_pass<double>(p, a, 4, 1, nullptr, w.x, w.t2, p->stream);
    if (!rc) rc = grad_accumulate((double*)dLdlogK, w.t1, w.t2, a == 0, p->npts, p->stream);
  }
  if (!rc) rc = grad_finish((double*)dLdlogK, Kd, p->npts, p->stream);
  if (!rc) rc = hip_check(hipStreamSynchronize(p->stream), "hipStreamSynchronize");
  if (rc) return rc;
  if (info) {
    cheb_solve_info inf{};
    inf.status = status;
    inf.matvecs = st.matvecs;
    inf.restarts = st.restarts;
    inf.history_used = st.hist_used;
    inf.relres_final = relres;
    inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *info = inf;
  }
  return status;
}

int cheb_picard(cheb_plan* plan, const void* K0, const void* f, const void* g_faces, void* u_inout, void* Kwork,
                double picard_tol, int32_t max_steps, const cheb_solve_opts* opts, cheb_solve_info* info,
                int32_t* steps) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!plan || !K0 || !f || !g_faces || !u_inout || !Kwork || max_steps < 1) {
    set_error("invalid argument");
    return CHEB_ERR_INVALID_ARG;
  }
  if (plan->prec == CHEB_F32) {
    set_error("Picard needs an FP64 or MIXED plan");
    return CHEB_ERR_UNSUPPORTED;
  }
  cheb_plan* p = plan;
  SolveParams sp = params_from(opts);
  // the previous iterate and the update live after the solver's own workspace
  const size_t base = solve_need(p, sp);
  const size_t fb = field_bytes(p->npts, sizeof(double));
  if (!p->ws || p->ws_bytes < base + 2 * fb) {
    set_error("workspace missing or too small (see cheb_plan_workspace_bytes)");
    return CHEB_ERR_WORKSPACE;
  }
  Scratch scr;
  if (p->prec == CHEB_MIXED) {
    MixedWS wm;
    carve_mixed(p, sp, (char*)p->ws, wm);
    scr = wm.sc;
  } else {
    SolveWS64 w64;
    carve64(p, sp, (char*)p->ws, w64);
    scr = w64.sc;
  }
  double* uold = (double*)((char*)p->ws + base);
  double* diff = (double*)((char*)p->ws + base + fb);
  int rc = CHEB_OK;
  if (!sp.warm) rc = fill<double>((double*)u_inout, 0.0, p->npts, p->stream);
  cheb_solve_opts o = opts ? *opts : cheb_solve_opts{};
  o.flags |= 1;
  cheb_solve_info tot{};
  int status = CHEB_NOT_CONVERGED;
  int nsteps = 0;
  for (int s = 0; s < max_steps && !rc; ++s) {
    rc = picard_coeff((double*)Kwork, (const double*)K0, (const double*)u_inout, p->npts, p->stream);
    if (!rc) rc = copy_scale<double>(uold, (const double*)u_inout, 1.0, p->npts, p->stream);
    if (rc) break;
    cheb_solve_info si{};
    const int r2 = cheb_solve(p, Kwork, f, g_faces, u_inout, &o, &si);
    if (r2 < 0) {
      rc = r2;
      break;
    }
    nsteps++;
    tot.matvecs += si.matvecs;
    tot.matvecs_f32 += si.matvecs_f32;
    tot.restarts += si.restarts;
    tot.ir_steps += si.ir_steps;
    tot.relres_final = si.relres_final;
    // relative update
    rc = copy_scale<double>(diff, (const double*)u_inout, 1.0, p->npts, p->stream);
    if (!rc) rc = axpby<double>(diff, uold, -1.0, 1.0, p->npts, p->stream);
    double dn = 0, un = 0;
    if (!rc) rc = vnorm<double>(p, diff, scr, &dn);
    if (!rc) rc = vnorm<double>(p, (const double*)u_inout, scr, &un);
    if (rc) break;
    if (sp.hist && s < sp.hist_len) sp.hist[s] = un > 0 ? dn / un : dn;
    if (r2 != CHEB_OK) {
      status = r2;
      break;
    }
    if (!(dn > picard_tol * un)) {
      status = CHEB_OK;
      break;
    }
  }
  if (rc) return rc;
  if (steps) *steps = nsteps;
  tot.status = status;
  tot.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  tot.history_used = nsteps < sp.hist_len ? nsteps : sp.hist_len;
  if (info) *info = tot;
  return status;
}

int cheb_newton_work_bytes(const cheb_plan* plan, size_t* bytes) {
  if (!plan || !bytes) {
    set_error("null argument");
    return CHEB_ERR_INVALID_ARG;
  }
  *bytes = kNewtonFields * field_bytes(plan->npts, sizeof(double)) + 256;
  return CHEB_OK;
}

int cheb_newton_residual(cheb_plan* plan, const void* K0, double alpha, const void* T, const void* f, void* r,
                         void* work) {
  if (!plan || !K0 || !T || !f || !r || !work) {
    set_error("null argument");
    return CHEB_ERR_INVALID_ARG;
  }
  int rc = newton_check_plan(plan);
  if (rc) return rc;
  cheb_plan* p = plan;
  NewtonWS w = newton_ws(p, work);
  rc = newton_linearise(p, (const double*)K0, alpha, (const double*)T, w);
  if (!rc) rc = newton_neg_residual(p, w, (const double*)T, (const double*)f, (double*)r);
  if (!rc) rc = copy_scale<double>((double*)r, (const double*)r, -1.0, p->npts, p->stream);
  if (!rc) rc = hip_check(hipStreamSynchronize(p->stream), "hipStreamSynchronize");
  return rc;
}

int cheb_newton_jacobian(cheb_plan* plan, const void* K0, double alpha, const void* T, const void* v, void* y,
                         void* work) {
  if (!plan || !K0 || !T || !v || !y || !work) {
    set_error("null argument");
    return CHEB_ERR_INVALID_ARG;
  }
  int rc = newton_check_plan(plan);
  if (rc) return rc;
  cheb_plan* p = plan;
  NewtonWS w = newton_ws(p, work);
  rc = newton_linearise(p, (const double*)K0, alpha, (const double*)T, w);
  if (!rc) rc = newton_jv(p, w, (const double*)v, (double*)y);
  if (!rc) rc = hip_check(hipStreamSynchronize(p->stream), "hipStreamSynchronize");
  return rc;
}

int cheb_newton(cheb_plan* plan, const void* K0, double alpha, const void* f, const void* g_faces, void* u_inout,
                void* work, double newton_tol, int32_t max_steps, const cheb_solve_opts* opts,
                cheb_solve_info* info, int32_t* steps, int32_t* mv_per_step) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!plan || !K0 || !f || !g_faces || !u_inout || !work || max_steps < 0 || !(newton_tol >= 0.0)) {
    set_error("invalid argument");
    return CHEB_ERR_INVALID_ARG;
  }
  int rc = newton_check_plan(plan);
  if (rc) return rc;
  cheb_plan* p = plan;
  const SolveParams sp = params_from(opts);
  if (sp.m < 1 || sp.m > 64 || sp.k < 0 || sp.k > 6) {
    set_error("inner_m must be in [1, 64] and outer_k in [0, 6]");
    return CHEB_ERR_INVALID_ARG;
  }
  SolveWS64 w64;
  const size_t need = carve64(p, sp, nullptr, w64);
  if (!p->ws || p->ws_bytes < need) {
    set_error("workspace missing or too small (see cheb_plan_workspace_bytes)");
    return CHEB_ERR_WORKSPACE;
  }
  carve64(p, sp, (char*)p->ws, w64);
  NewtonWS w = newton_ws(p, work);
  double* T = (double*)u_inout;
  hipStream_t s = p->stream;
  // reference scale: the residual of the cold start lift(0, g), whatever the
  // initial state, so that a warm start is judged on the same scale
  double rref = 0.0, rn = 0.0;
  int rc2 = fill<double>(w64.r, 0.0, p->npts, s);
  if (!rc2) rc2 = lift_full<double>(p, w64.r, (const double*)g_faces, s);
  if (!rc2) rc2 = newton_linearise(p, (const double*)K0, alpha, w64.r, w);
  if (!rc2) rc2 = newton_neg_residual(p, w, w64.r, (const double*)f, w64.bt);
  if (!rc2) rc2 = vnorm<double>(p, w64.bt, w64.sc, &rref);
  if (rc2) return rc2;
  if (!sp.warm) rc = copy_scale<double>(T, w64.r, 1.0, p->npts, s);
  else rc = lift_full<double>(p, T, (const double*)g_faces, s);
  if (!rc && sp.precond) rc = precond_setup(p);
  cheb_solve_info tot{};
  int status = CHEB_NOT_CONVERGED;
  int nsteps = 0;
  const double stop = newton_tol * rref;
  for (int m = 0; !rc; ++m) {
    rc = newton_linearise(p, (const double*)K0, alpha, T, w);
    if (!rc) rc = newton_neg_residual(p, w, T, (const double*)f, w64.bt);
    if (!rc) rc = vnorm<double>(p, w64.bt, w64.sc, &rn);
    if (rc) break;
    if (sp.hist && m < sp.hist_len) sp.hist[m] = rref > 0 ? rn / rref : 0.0;
    tot.history_used = m + 1 < sp.hist_len ? m + 1 : sp.hist_len;
    if (!(rn > stop)) {
      status = CHEB_OK;
      break;
    }
    if (m >= max_steps) break;
    double kc = 1.0;
    if (sp.precond) rc = mean_K<double>(p, w.k, w64.sc, &kc);
    if (!rc) rc = fill<double>(w64.x, 0.0, p->npts, s);
    if (rc) break;
    auto J = [&](const double* in, double* out) { return newton_jv(p, w, in, out); };
    auto Mi = [&](const double* in, double* out) {
      return precond_apply<double>(p, in, out, w64.kw.pa, w64.kw.pb, kc, false, s);
    };
    Stats st;
    double res = 0.0;
    // inexact Newton: the correction need not be more accurate than a tenth of
    // the outer target
    const double tol_lin = std::fmax(std::fmax(sp.rtol * rn, sp.atol), 0.1 * stop);
    const int r2 = lgmres<double>(p, J, w64.bt, w64.x, true, tol_lin, sp.maxiter, w64.kw,
                                  w64.sc, st, &res, rn, nullptr, 0, 0.0, sp.precond, Mi);
    if (r2 < 0) {
      rc = r2;
      break;
    }
    if (mv_per_step) mv_per_step[m] = st.matvecs;
    tot.matvecs += st.matvecs;
    tot.restarts += st.restarts;
    nsteps++;
    rc = mask_interior<double>(w64.x, p->g.n, s);
    if (!rc) rc = axpby<double>(T, w64.x, 1.0, 1.0, p->npts, s);
    if (!rc) rc = lift_full<double>(p, T, (const double*)g_faces, s);
  }
  if (!rc) rc = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
  if (rc) return rc;
  if (steps) *steps = nsteps;
  tot.status = status;
  tot.relres_final = rref > 0 ? rn / rref : 0.0;
  tot.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = tot;
  return status;
}

// Hierarchical refinement with its stopping rule (Section 2.3.3, Algorithm 4).
int cheb_refine(cheb_plan* const* plans, int32_t nlev, const void* const* K, const void* const* f,
                const void* const* g_faces, void* const* u, void* tmp, const cheb_solve_opts* opts, double tol,
                double* e_ref, int32_t* solved, cheb_solve_info* infos) {
  if (!plans || nlev < 1 || !K || !f || !g_faces || !u || (nlev > 1 && !tmp) || !(tol >= 0.0)) {
    set_error("invalid argument");
    return CHEB_ERR_INVALID_ARG;
  }
  for (int l = 0; l < nlev; ++l) {
    if (!plans[l] || !K[l] || !f[l] || !g_faces[l] || !u[l]) {
      set_error("null plan or field");
      return CHEB_ERR_INVALID_ARG;
    }
    if (l == 0) continue;
    const cheb_plan *pc = plans[l - 1], *pf = plans[l];
    if (pc->prec != pf->prec) {
      set_error("every level must have the same precision");
      return CHEB_ERR_INVALID_ARG;
    }
    for (int a = 0; a < 3; ++a) {
      if (pf->g.n[a] < pc->g.n[a] || pf->g.lo[a] != pc->g.lo[a] || pf->g.hi[a] != pc->g.hi[a]) {
        set_error("levels must share the box and grow in size");
        return CHEB_ERR_INVALID_ARG;
      }
    }
    for (int q = 0; q < 6; ++q) {
      if (pf->g.bc[q] != pc->g.bc[q] || pf->g.robin[q] != pc->g.robin[q]) {
        set_error("levels must share the face conditions");
        return CHEB_ERR_INVALID_ARG;
      }
    }
    if (pf->npts > plans[nlev - 1]->npts) {
      set_error("tmp holds the last level; the last level must be the largest");
      return CHEB_ERR_INVALID_ARG;
    }
  }
  cheb_solve_opts o{};
  if (opts) o = *opts;
  int worst = CHEB_OK;
  bool converged = false;
  for (int l = 0; l < nlev; ++l) {
    cheb_plan* p = plans[l];
    if (e_ref) e_ref[l] = std::nan("");
    if (solved) solved[l] = 0;
    cheb_solve_info inf{};
    if (l > 0) {
      // the modal prolongation of the previous level: the initial guess, or
      // -- once the refinement has converged -- the level's result
      int rc = cheb_prolong(plans[l - 1], p, u[l - 1], u[l], nullptr, nullptr);
      if (rc) return rc;
      if (converged) {
        rc = hip_check(hipStreamSynchronize(p->stream), "hipStreamSynchronize");
        if (rc) return rc;
        if (infos) infos[l] = inf;
        continue;
      }
      rc = p->prec == CHEB_F32 ? copy_scale<float>((float*)tmp, (const float*)u[l], 1.0, p->npts, p->stream)
                               : copy_scale<double>((double*)tmp, (const double*)u[l], 1.0, p->npts, p->stream);
      if (rc) return rc;
      o.flags |= 1;
    }
    const int st = cheb_solve(p, K[l], f[l], g_faces[l], u[l], &o, &inf);
    if (st < 0) return st;
    if (st > worst) worst = st;
    if (solved) solved[l] = 1;
    if (infos) infos[l] = inf;
    if (l > 0) {
      // e_ref = ||U_l - P U_{l-1}|| / ||U_l|| over the level's nodes
      double* part = (double*)p->ws;
      double* res = part + multidot_partials_len(p->npts, 1);
      int rc;
      if (p->prec == CHEB_F32) {
        rc = axpby<float>((float*)tmp, (const float*)u[l], -1.0, 1.0, p->npts, p->stream);
        if (!rc) rc = multidot<float>(nullptr, 0, 0, (const float*)tmp, p->npts, part, res, p->stream);
        if (!rc) rc = multidot<float>(nullptr, 0, 0, (const float*)u[l], p->npts, part, res + 1, p->stream);
      } else {
        rc = axpby<double>((double*)tmp, (const double*)u[l], -1.0, 1.0, p->npts, p->stream);
        if (!rc) rc = multidot<double>(nullptr, 0, 0, (const double*)tmp, p->npts, part, res, p->stream);
        if (!rc) rc = multidot<double>(nullptr, 0, 0, (const double*)u[l], p->npts, part, res + 1, p->stream);
      }
      double nn[2] = {0.0, 0.0};
      if (!rc) rc = readback(p, res, 2, nn);
      if (rc) return rc;
      const double e = nn[1] > 0 ? std::sqrt(nn[0] / nn[1]) : 0.0;
      if (e_ref) e_ref[l] = e;
      if (e <= tol) converged = true;
    }
  }
  return worst;
}

}  // extern "C"
