// Host-side internals of the C ABI: the plan object and the kernel launchers
// shared between translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/cheb.h"
#include "../../include/cheb_debug.h"
#include "pencil.h"

namespace cheb {

// Per-axis constants of the ascending, affinely scaled differentiation matrix.
struct AxisConst {
  int N;
  double L;
  double cscale;                 // -1 / (N L)
  double m00, m0N, mN0, mNN;     // corner entries
};

void set_error(const std::string& msg);
int hip_check(hipError_t e, const char* what);

// Launch facts of one kernel instantiation (resident workgroups, whether its
// LDS attribute is set), one slot per device, filled on the first launch on
// that device; concurrent first launches compute and store the same value.
constexpr int kMaxDevices = 64;
struct DeviceCache {
  std::atomic<int> v[kMaxDevices];
};

// ordinal of the calling thread's current device, within the cache's slots
inline int current_device(int* dev) {
  int rc = hip_check(hipGetDevice(dev), "hipGetDevice");
  if (!rc && (*dev < 0 || *dev >= kMaxDevices)) {
    set_error("device ordinal beyond the launch caches (64 devices)");
    rc = CHEB_ERR_UNSUPPORTED;
  }
  return rc;
}

// Workspace carving: fields padded to 256 bytes.
inline size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// fast-diagonalisation preconditioner factors of one axis (offsets into pc64/pc32)
struct PrecondAxis {
  int m;
  int split;  // centro-symmetric factors whose even and odd halves fill whole 16-row blocks
  int centro; // the axis' 1-D operator is centro-symmetric (the same face row at both ends)
  size_t off_V, off_Vi, off_lam;
  // matrix-core fragment tables (m <= 128): [0: the V^{-1} side, 1: the V side][transposed]
  size_t off_tab[2][2];  // an axis with the same 1-D problem as an earlier one shares its tables
};

}  // namespace cheb

struct cheb_plan {
  cheb_grid g;
  int prec;
  int device;  // HIP device current at creation (holds the plan's constants)
  hipStream_t stream;
  size_t npts;
  cheb::AxisConst ax[3];
  // device constants: per axis [row0 | rowN | cc weights | DCT twiddles W_2N^j (2N complex)],
  // slots of dconst_stride entries (the twiddles take 4 slots), f64 then f32
  double* dconst64;
  float* dconst32;
  size_t dconst_stride;  // entries per (axis, row) slot
  // host-pinned scratch for reductions and small coefficient vectors
  double* hpinned;
  size_t hpinned_len;
  void* ws;
  size_t ws_bytes;
  hipEvent_t ev;
  // fast-diagonalisation preconditioner (built on first use)
  int pc_ready;
  double* pc64;
  float* pc32;
  cheb::PrecondAxis pc_ax[3];
  // matrix-core route: split-product fragment tables of D (slot 0) and D^T (slot 1)
  int route;
  int dd_ok[3];
  size_t dd_off[3][2];
  int dense_var[3][2];  // tile shape of the matrix-core pass, [axis][f64, f32]
  int auto_fft[2];      // CHEB_ROUTE_AUTO resolved to the FFT route, [f64, f32] (autotuner)
  hipEvent_t kev[2];    // LGMRES: completion of the last two enqueued Arnoldi steps (created on first use)
  int kev_ok;
  // device flag the operator and preconditioner kernels check first (they do
  // nothing while it reads 0); set by LGMRES around each Arnoldi step so that
  // a step enqueued past the end of a restart cycle costs only its launches;
  // null otherwise
  const int* gate;
  double* dd64;
  float* dd32;
  // per-node Robin coefficients (cheb_plan_set_robin_nodes): packed faces in the
  // layout of g_faces, added to the grid's per-face coefficients, followed by
  // each axis' per-pencil end-block inverses (robin_inv_offset); FP64 and FP32
  // copies, null when unset.  rn_mean: the coefficients' face means.
  double* rn64;
  float* rn32;
  double rn_mean[6];
  // the two-axis launch's second output: one field (n0 n1 n2 values of the
  // plan's widest precision), allocated at creation when axes 0 and 1 have
  // the same N on the matrix-core route; null otherwise
  void* pair_buf;
};

namespace cheb {

// device constant pointers (axis a, slot s: 0 = row 0, 1 = row N, 2 = CC weights, 3 = twiddles)
constexpr int kConstSlots = 7;
inline const double* dconst64(const cheb_plan* p, int a, int s) {
  return p->dconst64 + (size_t)(kConstSlots * a + s) * p->dconst_stride;
}
inline const float* dconst32(const cheb_plan* p, int a, int s) {
  return p->dconst32 + (size_t)(kConstSlots * a + s) * p->dconst_stride;
}

// ---- operator passes (pass_f64.hip / pass_f32.hip) ----
// mode: 0 FULL, 1 REDUCED, 2 TRANSPOSE (reduced), 3 DERIV, 4 DERIV_T,
// 5 DERIV_ACC (y += D_a (K u) on interior nodes)
template <typename T>
int launch_axis_pass(const cheb_plan* p, int axis, int mode, int first, const T* K, const T* u, T* y,
                     hipStream_t s);

// full apply (z, y, x passes) in precision T
template <typename T>
int apply_t(const cheb_plan* p, const T* K, const T* u, T* y, int mode, hipStream_t s);

// ---- matrix-core route (dense_f64.hip / dense_f32.hip) ----
int dense_setup(cheb_plan* p);
struct DenseSys;
// batched reduced pass over the systems act[0..nact) of the table sys (same N,
// box and tile shape as `rep`); K, u, y are packed bases
template <typename T>
int launch_dense_batch(const cheb_plan* rep, int axis, int first, const T* K, const T* u, T* y,
                       const DenseSys* sys, const int* act, int nact, hipStream_t s);
// transpose: 0 reduced pass, 1 transposed reduced pass.  yadd: a second
// partial sum that the accumulating pass along the unit-stride axis (axis 2,
// first = 0) adds, and only that pass (null otherwise)
template <typename T>
int launch_dense_pass(const cheb_plan* p, int axis, int transpose, int first, const T* K, const T* u, T* y,
                      const T* yadd, hipStream_t s);
// the first passes along axes 0 and 1 in one launch, into y0 and y1; possible
// when all three axes take the matrix-core route, axes 0 and 1 have the same N
// and tile shape, and the plan holds pair_buf (dense_pair_ok)
template <typename T>
bool dense_pair_ok(const cheb_plan* p);
// y += D_a (c .* L v) on interior nodes (the Newton Jacobian's k'(T) term on
// the matrix-core route; FP64)
template <typename T>
int launch_dense_dacc(const cheb_plan* p, int axis, const T* c, const T* v, T* y, hipStream_t s);
// the Newton Jacobian's action in the two launches of the reduced apply (the
// c_a terms in the flux epilogues); CHEB_ERR_UNSUPPORTED when the plan cannot
template <typename T>
int launch_dense_jac(const cheb_plan* p, const T* K, const T* const* c, const T* v, T* y, hipStream_t s);
template <typename T>
int launch_dense_pair(const cheb_plan* p, int transpose, const T* K, const T* u, T* y0, T* y1, hipStream_t s);
// pi: 0 for the FP64 passes, 1 for the FP32 passes
inline bool use_dense(const cheb_plan* p, int axis, int pi) {
  if (!p->dd_ok[axis] || p->route == CHEB_ROUTE_FFT) return false;
  return p->route == CHEB_ROUTE_MATRIX || !p->auto_fft[pi];
}

// offset (entries) in rn64 / rn32 of axis a's per-pencil end-block inverses:
// 4 per pencil (i00, i0N, iN0, iNN of M^{-1}; 1 / m00 or 1 / mNN alone when the
// other end is Dirichlet), pencils in face numbering
inline size_t robin_inv_offset(const cheb_plan* p, int a) {
  return (size_t)face_offset(6, p->g.n) + 2 * (size_t)face_offset(2 * a, p->g.n);
}

// Robin coefficient of face f for the constant-coefficient preconditioner: the
// face's own plus the mean of its per-node part
inline double face_sigma(const cheb_plan* p, int f) { return p->g.robin[f] + (p->rn64 ? p->rn_mean[f] : 0.0); }

// Arnoldi: a second Gram-Schmidt pass runs when ||w - V h||^2 <= kReorthEta2 ||w||^2
constexpr double kReorthEta2 = 0.01;

// ---- device-resident LGMRES restart cycle (krylov.hip) ----
constexpr int kMaxKrylovCols = 70;  // inner_m + outer_k <= 64 + 6
// the part of the state the host reads back once per Arnoldi step
struct ArnoldiHead {
  double beta;      // ||r|| at the start of the cycle
  double est;       // residual estimate |g[jend]| after the last column
  double tol;       // absolute tolerance on ||r||
  double stall;     // stagnation factor (0: off)
  double bprev;     // beta of the previous cycle
  double inv_beta, hn, inv_hn;
  int active;       // 1 while the cycle is to continue
  int jend;         // columns built in this cycle
  int reorth;       // the cycle is paused at column jend for a second Gram-Schmidt pass
  int breakdown;
  int stagnated;    // beta > stall * bprev
  int direct;       // the next update forms v_{jend} (the last column was finalised and the cycle goes on)
  int pad_[2];
};
struct ArnoldiState : ArnoldiHead {
  double cs[kMaxKrylovCols], sn[kMaxKrylovCols], g[kMaxKrylovCols + 1], y[kMaxKrylovCols];
  double H[(kMaxKrylovCols + 1) * kMaxKrylovCols];  // row-major, rotated to upper triangular
};
int arnoldi_init(ArnoldiState* st, double tol, double stall, hipStream_t s);
// beta = sqrt(dots[0]); g = beta e_1; active = beta > tol and not stagnated
int arnoldi_begin(ArnoldiState* st, const double* dots, hipStream_t s);
// one Gram-Schmidt pass of Arnoldi step j against V_0..V_j and the Hessenberg
// column it gives (pass 0 while the cycle is active; pass 1, the
// re-orthogonalisation, only while pass 0 has paused the cycle for it: it
// first sets w <- w - V h0 with h0 the pass-0 coefficients); dots[0..j+1]
// receive the pass's coefficients and ||w||^2; partials:
// multidot_partials_len(npts, j + 1); host_head (pinned host memory, or null)
// receives the state's head once the column is done
template <typename T>
int gram_schmidt(const T* V, size_t ld, int j, T* w, size_t npts, const double* h0, double* partials,
                 double* dots, ArnoldiState* st, int pass, hipStream_t s, ArnoldiHead* host_head = nullptr);
// st->y = R^{-1} g over the cycle's columns
int arnoldi_solve(ArnoldiState* st, hipStream_t s);
template <typename T>
int scale_by(T* v, const double* dscale, size_t npts, hipStream_t s);  // v *= *dscale

// ---- vector kernels (blas.hip) ----
size_t multidot_partials_len(size_t npts, int nv);
// out[i] = <V_i, w> for i < nv, out[nv] = <w, w>  (double accumulation); with
// a gate, the kernels do nothing unless *gate != 0 when they run
template <typename T>
int multidot(const T* V, size_t ld, int nv, const T* w, size_t npts, double* partials, double* out,
             hipStream_t s, const int* gate = nullptr);
// out = (w - sum_i h_i V_i) * scale   (h on device, nv entries; out may alias w);
// dscale (device) replaces scale when given; gated as multidot
template <typename T>
int update_scale(const T* V, size_t ld, int nv, const double* h, const T* w, T* out, double scale,
                 size_t npts, hipStream_t s, const double* dscale = nullptr, const int* gate = nullptr);
// out (+)= sum_i c_i V_i  (c on device)
template <typename T>
int lincomb(const T* V, size_t ld, int nv, const double* c, T* out, int accumulate, size_t npts,
            hipStream_t s);
template <typename T>
int axpby(T* y, const T* x, double alpha, double beta, size_t npts, hipStream_t s);  // y = alpha x + beta y
template <typename T>
int copy_scale(T* y, const T* x, double alpha, size_t npts, hipStream_t s);  // y = alpha x
int cast_f64_f32(float* y, const double* x, double alpha, size_t npts, hipStream_t s);
int add_f32_to_f64(double* y, const float* x, double alpha, size_t npts, hipStream_t s);  // y += alpha x
template <typename T>
int fill(T* y, double v, size_t npts, hipStream_t s);
// y = (f - y) on interior nodes, 0 on boundary nodes
template <typename T>
int rhs_reduced(T* y, const T* f, const int* n, hipStream_t s);
template <typename T>
int mask_interior(T* y, const int* n, hipStream_t s);
// K-dependent pointwise kernels
int picard_coeff(double* K, const double* K0, const double* u, size_t npts, hipStream_t s);
// k = K0 / (1 + alpha T), kp = dk/dT
int newton_coeff(double* k, double* kp, const double* K0, const double* T, double alpha, size_t npts,
                 hipStream_t s);
int vmul(double* y, const double* a, const double* b, size_t npts, hipStream_t s);  // y = a * b (y may alias)
int grad_accumulate(double* g, const double* du, const double* dl, int first, size_t npts,
                    hipStream_t s);
int grad_finish(double* g, const double* K, size_t npts, hipStream_t s);
int check_positive_finite(const double* K, size_t npts, int* dflag, hipStream_t s);
int check_positive_finite_f32(const float* K, size_t npts, int* dflag, hipStream_t s);
// weighted sum  sum_ijk wx_i wy_j wz_k a_ijk b_ijk  -> partial sums, reduced into out[0]
int cc_dot(const double* a, const double* b, const double* wx, const double* wy, const double* wz,
           const int* n, double* partials, double* out, hipStream_t s);

// ---- lift kernels (lift.hip) ----
template <typename T>
int lift_full(const cheb_plan* p, T* U, const T* g_faces, hipStream_t s);     // x_r = G x_k + H g
template <typename T>
int lift_transpose(const cheb_plan* p, T* W, hipStream_t s);                  // W <- lift^T W (interior)

// ---- preconditioner (precond.hip) ----
int precond_setup(cheb_plan* p);
// out = M^{-1} in (or M^{-T} in); bufA/bufB: packed interior scratch (m0*m1*m2 each)
template <typename T>
int precond_apply(const cheb_plan* p, const T* in, T* out, T* bufA, T* bufB, double kc, bool transpose,
                  hipStream_t s);
// batched: members k < nmem of one group (same grid and face types as `rep`),
// packed fields at offs[k] (device), mean conductivity kc[sys[k]] (device);
// span = elements of the packed batch (every offs[k] + field size is within it)
template <typename T>
int precond_apply_batch(const cheb_plan* rep, const T* in, T* out, const long long* offs, const int* sys,
                        const double* kc, int nmem, size_t span, T* bufA, T* bufB, hipStream_t s);
// sum of all entries (double accumulation) into out[0]
template <typename T>
int vsum(const T* x, size_t npts, double* partials, double* out, hipStream_t s);

// ---- prolongation (prolong.hip) ----
template <typename T>
int prolong_t(const cheb_plan* pc, const cheb_plan* pf, const T* uc, T* uf, T* tmp1, T* tmp2,
              hipStream_t s);

}  // namespace cheb
