// Instantiation and dispatch of the matrix-core axis pass for one precision.
#pragma once

#include "dense_pass.h"
#include "internal.h"

namespace cheb {

// `kind` of the dispatch below: 0 reduced pass, 1 transposed reduced pass,
// kDenseDacc the Newton Jacobian's derivative pass (DENSE_DACC), kDenseJac the
// Jacobian's whole axis term (DENSE_JAC)
constexpr int kDenseDacc = 2;
constexpr int kDenseJac = 3;

// Persistent launch: as many workgroups as the device holds at once (resident
// workgroups per CU x CUs, queried once per kernel and device), at most one per
// tile.  A two-axis launch gives each axis half of them, a multiple of 8 (the
// kernel's segment bit is bit 3 of the workgroup index).
template <typename T, int NC, int MODE, bool FIRST, int V, bool CG>
static int launch_dense_inst(const DenseArgs<T>& a, hipStream_t s) {
  constexpr DenseDims S = dense_dims(NC, V);
  constexpr int lds = dense_lds_bytes<T>(NC, V, (MODE & DENSE_JAC) != 0);
  static_assert(lds <= 160 * 1024, "matrix-core tile exceeds LDS");
  static DeviceCache cache;
  int dev = 0;
  if (int rc = current_device(&dev)) return rc;
  int resident = cache.v[dev].load(std::memory_order_relaxed);
  if (resident == 0) {
    int cus = 0, per_cu = 0, rc = CHEB_OK;
    if (lds > 64 * 1024)
      rc = hip_check(hipFuncSetAttribute((const void*)k_dense_pass<T, NC, MODE, FIRST, V, CG>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, lds),
                     "matrix-core pass LDS attribute");
    if (!rc) rc = hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "CU count");
    if (!rc)
      rc = hip_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_dense_pass<T, NC, MODE, FIRST, V, CG>,
                                                                  64 * S.NW, lds),
                     "occupancy query");
    if (rc) return rc;
    resident = (cus > 0 ? cus : 1) * (per_cu > 0 ? per_cu : 1);
    cache.v[dev].store(resident, std::memory_order_relaxed);
  }
  auto tiles_of = [&](int axis) {
    const int ta = axis == 0 ? a.n[1] : a.n[0], tb = axis == 2 ? a.n[1] : a.n[2];
    return ((ta - 2) * (tb - 2) + S.C - 1) / S.C * (a.sys ? a.nact : 1);
  };
  int grid;
  if (a.nseg == 2) {
    const int t0 = tiles_of(a.ax[0].axis), t1 = tiles_of(a.ax[1].axis);
    const int need = ((t0 > t1 ? t0 : t1) + 7) / 8 * 8;
    int half = resident / 2 / 8 * 8;
    if (need < half) half = need;
    if (half < 8) half = 8;
    grid = 2 * half;
  } else {
    const int tiles = tiles_of(a.ax[0].axis);
    grid = tiles < resident ? (tiles > 0 ? tiles : 1) : resident;
  }
  hipLaunchKernelGGL((k_dense_pass<T, NC, MODE, FIRST, V, CG>), dim3(grid), dim3(64 * S.NW), lds, s, a);
  return hip_check(hipGetLastError(), "matrix-core pass launch");
}

template <typename T, int NC, int V, bool CG, bool RN>
static int launch_dense_c(const DenseArgs<T>& a, int first, int kind, hipStream_t s) {
  constexpr int MR = DENSE_REDUCED | (RN ? DENSE_NODE : 0), MT = DENSE_TRANSPOSE | (RN ? DENSE_NODE : 0);
  if (kind == kDenseDacc) {
    // the Newton Jacobian's accumulating derivative pass (FP64 plans only)
    if constexpr (sizeof(T) == sizeof(double))
      return launch_dense_inst<T, NC, MR | DENSE_DACC, false, V, CG>(a, s);
    set_error("matrix-core derivative pass: FP64 only");
    return CHEB_ERR_UNSUPPORTED;
  }
  if (kind == kDenseJac) {
    // the Newton Jacobian's axis terms (FP64 plans, 4-wave tiles)
    if constexpr (sizeof(T) == sizeof(double) && V == 1)
      return first ? launch_dense_inst<T, NC, MR | DENSE_JAC, true, V, CG>(a, s)
                   : launch_dense_inst<T, NC, MR | DENSE_JAC, false, V, CG>(a, s);
    set_error("matrix-core Jacobian pass: FP64 and tile shape 1 only");
    return CHEB_ERR_UNSUPPORTED;
  }
  if (first)
    return kind ? launch_dense_inst<T, NC, MT, true, V, CG>(a, s) : launch_dense_inst<T, NC, MR, true, V, CG>(a, s);
  return kind ? launch_dense_inst<T, NC, MT, false, V, CG>(a, s) : launch_dense_inst<T, NC, MR, false, V, CG>(a, s);
}

template <typename T, int NC, int V, bool RN>
static int launch_dense_v(const DenseArgs<T>& a, int first, int kind, hipStream_t s) {
  return a.ax[0].axis == 2 ? launch_dense_c<T, NC, V, true, RN>(a, first, kind, s)
                           : launch_dense_c<T, NC, V, false, RN>(a, first, kind, s);
}

template <typename T, int NC, bool RN>
static int launch_dense_n(const DenseArgs<T>& a, int first, int kind, int variant, hipStream_t s) {
  return variant == 1 ? launch_dense_v<T, NC, 1, RN>(a, first, kind, s)
                      : launch_dense_v<T, NC, 0, RN>(a, first, kind, s);
}

// every N and tile shape of the pass, with (RN) or without per-node Robin
// inverses; the two sets are instantiated in separate files (dense_f64.hip /
// dense_f64_rn.hip and the FP32 pair) so that they compile in parallel
template <typename T, bool RN>
int launch_dense_rn(const DenseArgs<T>& a, int N, int first, int kind, int variant, hipStream_t s) {
  switch (N) {
    case 16: return launch_dense_n<T, 16, RN>(a, first, kind, variant, s);
    case 32: return launch_dense_n<T, 32, RN>(a, first, kind, variant, s);
    case 48: return launch_dense_n<T, 48, RN>(a, first, kind, variant, s);
    case 64: return launch_dense_n<T, 64, RN>(a, first, kind, variant, s);
    case 96: return launch_dense_n<T, 96, RN>(a, first, kind, variant, s);
    case 128: return launch_dense_n<T, 128, RN>(a, first, kind, variant, s);
    default: set_error("matrix-core pass: unsupported N"); return CHEB_ERR_UNSUPPORTED;
  }
}
extern template int launch_dense_rn<double, true>(const DenseArgs<double>&, int, int, int, int, hipStream_t);
extern template int launch_dense_rn<float, true>(const DenseArgs<float>&, int, int, int, int, hipStream_t);

template <typename T>
static const T* dense_tab(const cheb_plan* p, int axis, int transpose);
template <>
inline const double* dense_tab<double>(const cheb_plan* p, int axis, int transpose) {
  return p->dd64 + p->dd_off[axis][transpose];
}
template <>
inline const float* dense_tab<float>(const cheb_plan* p, int axis, int transpose) {
  return p->dd32 + p->dd_off[axis][transpose];
}

// the launch fields of one axis: tables, lift entries, per-node inverses, output
template <typename T>
static DenseAxis<T> dense_axis(const cheb_plan* p, int axis, int transpose, bool batch, T* y) {
  DenseAxis<T> x;
  x.tab = dense_tab<T>(p, axis, transpose);
  const size_t slot0 = (size_t)(kConstSlots * axis) * p->dconst_stride;
  const size_t slotN = (size_t)(kConstSlots * axis + 1) * p->dconst_stride;
  if (sizeof(T) == sizeof(double)) {
    x.drow0 = (const T*)(p->dconst64 + slot0);
    x.drowN = (const T*)(p->dconst64 + slotN);
  } else {
    x.drow0 = (const T*)(p->dconst32 + slot0);
    x.drowN = (const T*)(p->dconst32 + slotN);
  }
  x.y = y;
  x.c = nullptr;
  x.axis = axis;
  {
    const double m00 = p->ax[axis].m00, m0N = p->ax[axis].m0N, mN0 = p->ax[axis].mN0, mNN = p->ax[axis].mNN;
    // entries that belong to a Dirichlet end are never used; keep them finite
    const double det = m00 * mNN - m0N * mN0, id = det != 0.0 ? 1.0 / det : 0.0;
    x.i00 = T(mNN * id);
    x.i0N = T(-m0N * id);
    x.iN0 = T(-mN0 * id);
    x.iNN = T(m00 * id);
    x.r00 = T(m00 != 0.0 ? 1.0 / m00 : 0.0);
    x.rNN = T(mNN != 0.0 ? 1.0 / mNN : 0.0);
  }
  x.rinv = nullptr;
  if (!batch && p->rn64) {
    if (sizeof(T) == sizeof(double)) x.rinv = (const T*)(p->rn64 + robin_inv_offset(p, axis));
    else x.rinv = (const T*)(p->rn32 + robin_inv_offset(p, axis));
  }
  return x;
}

template <typename T>
static DenseArgs<T> dense_args(const cheb_plan* p, const T* K, const T* u, const DenseSys* sys, const int* act,
                               int nact) {
  DenseArgs<T> a;
  a.gate = sys ? nullptr : p->gate;
  a.u = u;
  a.K = K;
  a.sys = sys;
  a.act = act;
  a.nact = nact;
  for (int i = 0; i < 3; ++i) a.n[i] = p->g.n[i];
  a.bcmask = bc_mask(p->g.bc);
  a.nseg = 1;
  a.yadd = nullptr;
  return a;
}

template <typename T>
static int launch_dense_common(const cheb_plan* p, int axis, int transpose, int first, const T* K, const T* u,
                               T* y, const T* yadd, const DenseSys* sys, const int* act, int nact, hipStream_t s) {
  // the accumulating pass along the unit-stride axis is the last pass of a
  // two-axis apply, and its kernel always adds yadd
  if ((axis == 2 && !first) != (yadd != nullptr)) {
    set_error("matrix-core pass: the second partial sum goes with the accumulating unit-stride pass only");
    return CHEB_ERR_INVALID_ARG;
  }
  DenseArgs<T> a = dense_args<T>(p, K, u, sys, act, nact);
  a.ax[0] = dense_axis<T>(p, axis, transpose, sys != nullptr, y);
  a.ax[1] = a.ax[0];
  a.yadd = yadd;
  const int variant = p->dense_var[axis][sizeof(T) == sizeof(double) ? 0 : 1];
  return a.ax[0].rinv ? launch_dense_rn<T, true>(a, p->ax[axis].N, first, transpose, variant, s)
                      : launch_dense_rn<T, false>(a, p->ax[axis].N, first, transpose, variant, s);
}

template <typename T>
int launch_dense_pass(const cheb_plan* p, int axis, int transpose, int first, const T* K, const T* u, T* y,
                      const T* yadd, hipStream_t s) {
  return launch_dense_common<T>(p, axis, transpose, first, K, u, y, yadd, nullptr, nullptr, 0, s);
}

// y = sum_a D_a (K .* D_a L v + c_a .* L v) on interior nodes, 0 on boundary
// nodes: the Newton Jacobian's action (the reduced operator at K plus the
// k'(T) terms) in the two launches of the reduced apply, the c_a term added
// in each flux epilogue.  CHEB_ERR_UNSUPPORTED when the plan's passes cannot
// take that form (FP64 only; all axes on the matrix-core route with tile shape
// 1, the x and y passes sharing a launch); the caller then takes the separate
// passes.
template <typename T>
int launch_dense_jac(const cheb_plan* p, const T* K, const T* const* c, const T* v, T* y, hipStream_t s) {
  if (sizeof(T) != sizeof(double) || !dense_pair_ok<T>(p) || p->dense_var[0][0] != 1 || p->dense_var[2][0] != 1)
    return CHEB_ERR_UNSUPPORTED;
  T* y1 = (T*)p->pair_buf;
  DenseArgs<T> a = dense_args<T>(p, K, v, nullptr, nullptr, 0);
  a.nseg = 2;
  a.ax[0] = dense_axis<T>(p, 0, 0, false, y);
  a.ax[1] = dense_axis<T>(p, 1, 0, false, y1);
  a.ax[0].c = c[0];
  a.ax[1].c = c[1];
  int rc = a.ax[0].rinv ? launch_dense_rn<T, true>(a, p->ax[0].N, 1, kDenseJac, 1, s)
                        : launch_dense_rn<T, false>(a, p->ax[0].N, 1, kDenseJac, 1, s);
  if (rc) return rc;
  DenseArgs<T> z = dense_args<T>(p, K, v, nullptr, nullptr, 0);
  z.ax[0] = dense_axis<T>(p, 2, 0, false, y);
  z.ax[0].c = c[2];
  z.ax[1] = z.ax[0];
  z.yadd = y1;
  return z.ax[0].rinv ? launch_dense_rn<T, true>(z, p->ax[2].N, 0, kDenseJac, 1, s)
                      : launch_dense_rn<T, false>(z, p->ax[2].N, 0, kDenseJac, 1, s);
}

// y += D_a (c .* L v) on the interior nodes of interior-transverse pencils
// along axis a (L v: v's interior values with the end values of the
// homogeneous lift), accumulating: the matrix-core form of the FFT route's
// MODE_DERIV_ACC pass
template <typename T>
int launch_dense_dacc(const cheb_plan* p, int axis, const T* c, const T* v, T* y, hipStream_t s) {
  DenseArgs<T> a = dense_args<T>(p, c, v, nullptr, nullptr, 0);
  a.ax[0] = dense_axis<T>(p, axis, 0, false, y);
  a.ax[1] = a.ax[0];
  const int variant = p->dense_var[axis][sizeof(T) == sizeof(double) ? 0 : 1];
  return a.ax[0].rinv ? launch_dense_rn<T, true>(a, p->ax[axis].N, 0, kDenseDacc, variant, s)
                      : launch_dense_rn<T, false>(a, p->ax[axis].N, 0, kDenseDacc, variant, s);
}

template <typename T>
bool dense_pair_ok(const cheb_plan* p) {
  const int pi = sizeof(T) == sizeof(double) ? 0 : 1;
  return p->pair_buf && use_dense(p, 0, pi) && use_dense(p, 1, pi) && use_dense(p, 2, pi) &&
         p->ax[0].N == p->ax[1].N && p->dense_var[0][pi] == p->dense_var[1][pi];
}

template <typename T>
int launch_dense_pair(const cheb_plan* p, int transpose, const T* K, const T* u, T* y0, T* y1, hipStream_t s) {
  if (!dense_pair_ok<T>(p)) {
    set_error("matrix-core pass: axes 0 and 1 cannot share a launch");
    return CHEB_ERR_INVALID_ARG;
  }
  DenseArgs<T> a = dense_args<T>(p, K, u, nullptr, nullptr, 0);
  a.nseg = 2;
  a.ax[0] = dense_axis<T>(p, 0, transpose, false, y0);
  a.ax[1] = dense_axis<T>(p, 1, transpose, false, y1);
  const int variant = p->dense_var[0][sizeof(T) == sizeof(double) ? 0 : 1];
  return a.ax[0].rinv ? launch_dense_rn<T, true>(a, p->ax[0].N, 1, transpose, variant, s)
                      : launch_dense_rn<T, false>(a, p->ax[0].N, 1, transpose, variant, s);
}

template <typename T>
int launch_dense_batch(const cheb_plan* rep, int axis, int first, const T* K, const T* u, T* y,
                       const DenseSys* sys, const int* act, int nact, hipStream_t s) {
  if (nact <= 0) return CHEB_OK;
  return launch_dense_common<T>(rep, axis, 0, first, K, u, y, nullptr, sys, act, nact, s);
}

}  // namespace cheb
