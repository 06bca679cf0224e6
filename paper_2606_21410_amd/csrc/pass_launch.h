// Instantiation and dispatch of the axis-pass kernel for one precision.
#pragma once

#include "internal.h"
#include "pass_kernel.h"

namespace cheb {

template <typename T, int NC, int MODE>
static int launch_pass_inst(const PassArgs<T>& a, hipStream_t s) {
  const PassLayout lay = pass_layout<T>(NC, a.N);
  constexpr int P = pass_pencils(NC);
  constexpr int NT = pass_threads(NC);
  const int tiles = (a.npencils + P - 1) / P;
  if (lay.bytes > 160 * 1024) {
    set_error("axis pass tile does not fit in LDS");
    return CHEB_ERR_UNSUPPORTED;
  }
  static DeviceCache attr_set;  // 1 once the LDS attribute is set on the device
  int dev = 0;
  if (lay.bytes > 64 * 1024) {
    if (int rc = current_device(&dev)) return rc;
  }
  if (lay.bytes > 64 * 1024 && !attr_set.v[dev].load(std::memory_order_relaxed)) {
    hipError_t e = hipFuncSetAttribute((const void*)k_axis_pass<T, NC, MODE>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lay.bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      set_error("axis pass tile needs more LDS than the device grants");
      return CHEB_ERR_UNSUPPORTED;
    }
    attr_set.v[dev].store(1, std::memory_order_relaxed);
  }
  hipLaunchKernelGGL((k_axis_pass<T, NC, MODE>), dim3(tiles), dim3(NT), lay.bytes, s, a);
  return hip_check(hipGetLastError(), "axis pass launch");
}

template <typename T, int NC>
static int launch_pass_mode(const PassArgs<T>& a, int mode, hipStream_t s) {
  switch (mode) {
    case MODE_FULL: return launch_pass_inst<T, NC, MODE_FULL>(a, s);
    case MODE_REDUCED: return launch_pass_inst<T, NC, MODE_REDUCED>(a, s);
    case MODE_TRANSPOSE: return launch_pass_inst<T, NC, MODE_TRANSPOSE>(a, s);
    case MODE_DERIV: return launch_pass_inst<T, NC, MODE_DERIV>(a, s);
    case MODE_DERIV_T: return launch_pass_inst<T, NC, MODE_DERIV_T>(a, s);
    case MODE_DERIV_ACC: return launch_pass_inst<T, NC, MODE_DERIV_ACC>(a, s);
    default: set_error("bad pass mode"); return CHEB_ERR_INVALID_ARG;
  }
}

template <typename T>
static int dispatch_pass(const PassArgs<T>& a, int mode, hipStream_t s) {
  switch (a.N) {
    case 4: return launch_pass_mode<T, 4>(a, mode, s);
    case 8: return launch_pass_mode<T, 8>(a, mode, s);
    case 12: return launch_pass_mode<T, 12>(a, mode, s);
    case 16: return launch_pass_mode<T, 16>(a, mode, s);
    case 24: return launch_pass_mode<T, 24>(a, mode, s);
    case 32: return launch_pass_mode<T, 32>(a, mode, s);
    case 48: return launch_pass_mode<T, 48>(a, mode, s);
    case 64: return launch_pass_mode<T, 64>(a, mode, s);
    case 96: return launch_pass_mode<T, 96>(a, mode, s);
    case 128: return launch_pass_mode<T, 128>(a, mode, s);
    case 192: return launch_pass_mode<T, 192>(a, mode, s);
    case 256: return launch_pass_mode<T, 256>(a, mode, s);
    case 384: return launch_pass_mode<T, 384>(a, mode, s);
    case 512: return launch_pass_mode<T, 512>(a, mode, s);
    default: return launch_pass_mode<T, 0>(a, mode, s);
  }
}

template <typename T>
static const T* drow(const cheb_plan* p, int a, int slot);
template <>
inline const double* drow<double>(const cheb_plan* p, int a, int slot) { return dconst64(p, a, slot); }
template <>
inline const float* drow<float>(const cheb_plan* p, int a, int slot) { return dconst32(p, a, slot); }

template <typename T>
static const T* robin_nodes(const cheb_plan* p);
template <>
inline const double* robin_nodes<double>(const cheb_plan* p) { return p->rn64; }
template <>
inline const float* robin_nodes<float>(const cheb_plan* p) { return p->rn32; }

template <typename T>
int launch_axis_pass(const cheb_plan* p, int axis, int mode, int first, const T* K, const T* u, T* y,
                     hipStream_t s) {
  if ((mode == MODE_REDUCED || mode == MODE_TRANSPOSE) && use_dense(p, axis, sizeof(T) == sizeof(double) ? 0 : 1))
    return launch_dense_pass<T>(p, axis, mode == MODE_TRANSPOSE ? 1 : 0, first, K, u, y, nullptr, s);
  if constexpr (sizeof(T) == sizeof(double)) {
    if (mode == MODE_DERIV_ACC && !first && use_dense(p, axis, 0)) return launch_dense_dacc<T>(p, axis, K, u, y, s);
  }
  PassArgs<T> a;
  a.gate = p->gate;
  a.u = u;
  a.K = K;
  a.y = y;
  a.drow0 = drow<T>(p, axis, 0);
  a.drowN = drow<T>(p, axis, 1);
  a.twg = drow<T>(p, axis, 3);
  for (int i = 0; i < 3; ++i) a.n[i] = p->g.n[i];
  a.bcmask = bc_mask(p->g.bc);
  a.axis = axis;
  a.N = p->ax[axis].N;
  a.first = first;
  a.cscale = T(p->ax[axis].cscale);
  a.m00 = T(p->ax[axis].m00);
  a.m0N = T(p->ax[axis].m0N);
  a.mN0 = T(p->ax[axis].mN0);
  a.mNN = T(p->ax[axis].mNN);
  a.slo = T(p->g.robin[2 * axis]);
  a.shi = T(p->g.robin[2 * axis + 1]);
  a.rnode = robin_nodes<T>(p);
  a.rlo = (int)face_offset(2 * axis, a.n);
  a.rhi = (int)face_offset(2 * axis + 1, a.n);
  a.npencils = pencil_count(axis, a.n);
  return dispatch_pass<T>(a, mode, s);
}

template <typename T>
int apply_t(const cheb_plan* p, const T* K, const T* u, T* y, int mode, hipStream_t s) {
  if ((mode == MODE_REDUCED || mode == MODE_TRANSPOSE) && dense_pair_ok<T>(p)) {
    // matrix-core route: the x and y passes in one launch (x into y, y into
    // the plan's second buffer; each initialises every row it owns), then the
    // z pass adds both to its own
    const int tr = mode == MODE_TRANSPOSE ? 1 : 0;
    T* y1 = (T*)p->pair_buf;
    int rc = launch_dense_pair<T>(p, tr, K, u, y, y1, s);
    if (rc) return rc;
    return launch_dense_pass<T>(p, 2, tr, 0, K, u, y, y1, s);
  }
  // z pass first (it initialises every row it owns), then y, then x
  int rc = launch_axis_pass<T>(p, 2, mode, 1, K, u, y, s);
  if (rc) return rc;
  rc = launch_axis_pass<T>(p, 1, mode, 0, K, u, y, s);
  if (rc) return rc;
  return launch_axis_pass<T>(p, 0, mode, 0, K, u, y, s);
}

}  // namespace cheb
