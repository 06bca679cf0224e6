// Modal prolongation (Section 2.3.3): along each axis, the DCT-I of the coarse
// pencil gives its Chebyshev coefficients, the coefficients are zero-padded to
// the fine degree and the fine pencil is their cosine sum at the fine CGL
// nodes.  z, then y, then x: (nc,nc,nc) -> (nc,nc,nf) -> (nc,nf,nf) -> (nf,nf,nf).
// Both transforms are evaluated as direct cosine sums from LDS tables; the
// prolongation runs once per refinement level, far off the solver's hot loop.
#include <cmath>
#include <mutex>

#include "internal.h"

namespace cheb {

namespace {

constexpr int kPP = 16;    // pencils per tile
constexpr int kPT = 256;   // threads

__device__ __forceinline__ void pencil_geom(int axis, int p, const int* n, long long* base, long long* stride) {
  if (axis == 2) {
    *base = (long long)p * n[2];
    *stride = 1;
  } else if (axis == 1) {
    const int ia = p / n[2], ib = p - ia * n[2];
    *base = (long long)ia * n[1] * n[2] + ib;
    *stride = n[2];
  } else {
    *base = p;
    *stride = (long long)n[1] * n[2];
  }
}

template <typename T>
__global__ __launch_bounds__(kPT) void k_prolong_axis(const T* __restrict__ src, T* __restrict__ dst, int axis,
                                                     int s0, int s1, int s2, int d0, int d1, int d2) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int ns[3] = {s0, s1, s2}, nd[3] = {d0, d1, d2};
  const int Nc = ns[axis] - 1, Nf = nd[axis] - 1;
  const int nc = Nc + 1, nf = Nf + 1;
  const int npen = axis == 2 ? s0 * s1 : axis == 1 ? s0 * s2 : s1 * s2;
  double* cc = (double*)smem;            // cos(pi j / Nc), j < 2 Nc
  double* cf = cc + 2 * Nc;              // cos(pi j / Nf), j < 2 Nf
  double* su = cf + 2 * Nf;              // kPP x nc pencil values
  double* sb = su + kPP * nc;            // kPP x nc scaled coefficients
  const int tid = threadIdx.x;
  const int p0 = blockIdx.x * kPP;
  for (int j = tid; j < 2 * Nc; j += kPT) cc[j] = cospi(double(j) / double(Nc));
  for (int j = tid; j < 2 * Nf; j += kPT) cf[j] = cospi(double(j) / double(Nf));
  for (int e = tid; e < kPP * nc; e += kPT) {
    const int m = e / kPP, pl = e - m * kPP;
    const int p = p0 + pl;
    double v = 0.0;
    if (p < npen) {
      long long b, st;
      pencil_geom(axis, p, ns, &b, &st);
      v = double(src[b + m * st]);
    }
    su[pl * nc + m] = v;
  }
  __syncthreads();
  // coefficients b_k = X_k / (2 Nc) (k < Nc), b_Nc = X_Nc / (4 Nc) when padding
  for (int e = tid; e < kPP * nc; e += kPT) {
    const int pl = e / nc, k = e - pl * nc;
    const double* u = su + pl * nc;
    double acc = u[0] + ((k & 1) ? -u[Nc] : u[Nc]);
    int idx = 0;
    for (int m = 1; m < Nc; ++m) {
      idx += k;
      if (idx >= 2 * Nc) idx -= 2 * Nc;
      acc += 2.0 * u[m] * cc[idx];
    }
    double sc = 1.0 / (2.0 * Nc);
    if (k == Nc && Nf > Nc) sc *= 0.5;
    if (Nf == Nc && (k == 0 || k == Nc)) sc = 1.0 / (2.0 * Nc);
    sb[pl * nc + k] = acc * sc;
  }
  __syncthreads();
  // fine values: b_0 + 2 sum_{k=1}^{Nc} b_k cos(pi k m / Nf)  (b_Nf term when Nf == Nc)
  for (int e = tid; e < kPP * nf; e += kPT) {
    const int m = e / kPP, pl = e - m * kPP;
    const int p = p0 + pl;
    if (p >= npen) continue;
    const double* b = sb + pl * nc;
    double acc = b[0];
    const int kend = (Nf == Nc) ? Nc - 1 : Nc;
    int idx = 0;
    for (int k = 1; k <= kend; ++k) {
      idx += m;
      if (idx >= 2 * Nf) idx -= 2 * Nf;
      acc += 2.0 * b[k] * cf[idx];
    }
    if (Nf == Nc) acc += ((m & 1) ? -b[Nc] : b[Nc]);
    long long bd, sd;
    pencil_geom(axis, p, nd, &bd, &sd);
    dst[bd + m * sd] = T(acc);
  }
}

}  // namespace

template <typename T>
int prolong_t(const cheb_plan* pc, const cheb_plan* pf, const T* uc, T* uf, T* tmp1, T* tmp2, hipStream_t s) {
  int cur[3] = {pc->g.n[0], pc->g.n[1], pc->g.n[2]};
  const T* in = uc;
  for (int step = 0; step < 3; ++step) {
    const int axis = 2 - step;
    int nxt[3] = {cur[0], cur[1], cur[2]};
    nxt[axis] = pf->g.n[axis];
    T* out = step == 2 ? uf : (step == 0 ? tmp1 : tmp2);
    const int npen = axis == 2 ? cur[0] * cur[1] : axis == 1 ? cur[0] * cur[2] : cur[1] * cur[2];
    const int Nc = cur[axis] - 1, Nf = nxt[axis] - 1;
    const size_t lds = (size_t)(2 * Nc + 2 * Nf + 2 * kPP * (Nc + 1)) * sizeof(double);
    if (lds > 64 * 1024) {
      if (hipFuncSetAttribute((const void*)k_prolong_axis<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds) != hipSuccess) {
        (void)hipGetLastError();
        set_error("prolongation tile needs more LDS than the device grants");
        return CHEB_ERR_UNSUPPORTED;
      }
    }
    hipLaunchKernelGGL(k_prolong_axis<T>, dim3((npen + kPP - 1) / kPP), dim3(kPT), lds, s, in, out, axis,
                       cur[0], cur[1], cur[2], nxt[0], nxt[1], nxt[2]);
    int rc = hip_check(hipGetLastError(), "prolongation");
    if (rc) return rc;
    in = out;
    for (int i = 0; i < 3; ++i) cur[i] = nxt[i];
  }
  return CHEB_OK;
}

template int prolong_t<double>(const cheb_plan*, const cheb_plan*, const double*, double*, double*, double*,
                               hipStream_t);
template int prolong_t<float>(const cheb_plan*, const cheb_plan*, const float*, float*, float*, float*,
                              hipStream_t);

}  // namespace cheb

using namespace cheb;

extern "C" int cheb_prolong(const cheb_plan* coarse, const cheb_plan* fine, const void* u_c, void* u_f,
                            const void* u_f_solved, double* e_ref) {
  if (!coarse || !fine || !u_c || !u_f || u_c == u_f) {
    set_error("invalid argument");
    return CHEB_ERR_INVALID_ARG;
  }
  if (coarse->prec != fine->prec) {
    set_error("coarse and fine plans must have the same precision");
    return CHEB_ERR_INVALID_ARG;
  }
  for (int a = 0; a < 3; ++a) {
    if (fine->g.n[a] < coarse->g.n[a]) {
      set_error("fine grid must not be smaller than the coarse grid");
      return CHEB_ERR_INVALID_ARG;
    }
    if (std::fabs(fine->g.lo[a] - coarse->g.lo[a]) > 0 || std::fabs(fine->g.hi[a] - coarse->g.hi[a]) > 0) {
      set_error("coarse and fine plans must describe the same box");
      return CHEB_ERR_INVALID_ARG;
    }
  }
  cheb_plan* pf = const_cast<cheb_plan*>(fine);
  const size_t esz = fine->prec == CHEB_F32 ? sizeof(float) : sizeof(double);
  const size_t fb = round_up(fine->npts * esz, 256);
  const size_t plen = multidot_partials_len(fine->npts, 1);
  const size_t need = 2 * fb + round_up((plen + 16) * sizeof(double), 256);
  if (!pf->ws || pf->ws_bytes < need) {
    set_error("prolongation needs the fine plan's workspace");
    return CHEB_ERR_WORKSPACE;
  }
  char* ws = (char*)pf->ws;
  int rc;
  if (fine->prec == CHEB_F32)
    rc = prolong_t<float>(coarse, fine, (const float*)u_c, (float*)u_f, (float*)ws, (float*)(ws + fb),
                          pf->stream);
  else
    rc = prolong_t<double>(coarse, fine, (const double*)u_c, (double*)u_f, (double*)ws, (double*)(ws + fb),
                           pf->stream);
  if (rc) return rc;
  if (u_f_solved && e_ref) {
    double* part = (double*)(ws + 2 * fb);
    double* res = part + plen;
    if (fine->prec == CHEB_F32) {
      float* d = (float*)ws;
      rc = copy_scale<float>(d, (const float*)u_f_solved, 1.0, fine->npts, pf->stream);
      if (!rc) rc = axpby<float>(d, (const float*)u_f, -1.0, 1.0, fine->npts, pf->stream);
      if (!rc) rc = multidot<float>(nullptr, 0, 0, d, fine->npts, part, res, pf->stream);
      if (!rc) rc = multidot<float>(nullptr, 0, 0, (const float*)u_f_solved, fine->npts, part, res + 1, pf->stream);
    } else {
      double* d = (double*)ws;
      rc = copy_scale<double>(d, (const double*)u_f_solved, 1.0, fine->npts, pf->stream);
      if (!rc) rc = axpby<double>(d, (const double*)u_f, -1.0, 1.0, fine->npts, pf->stream);
      if (!rc) rc = multidot<double>(nullptr, 0, 0, d, fine->npts, part, res, pf->stream);
      if (!rc)
        rc = multidot<double>(nullptr, 0, 0, (const double*)u_f_solved, fine->npts, part, res + 1, pf->stream);
    }
    if (!rc)
      rc = hip_check(hipMemcpyAsync(pf->hpinned, res, 2 * sizeof(double), hipMemcpyDeviceToHost, pf->stream),
                     "hipMemcpyAsync");
    if (!rc) rc = hip_check(hipStreamSynchronize(pf->stream), "hipStreamSynchronize");
    if (rc) return rc;
    *e_ref = pf->hpinned[1] > 0 ? std::sqrt(pf->hpinned[0] / pf->hpinned[1]) : 0.0;
  }
  return CHEB_OK;
}

// ---- allocation-free prolongation ------------------------------------------
// The two intermediate fields of the three axis passes live in a file-scope
// device array instead of the fine plan's workspace.  Every GPU that runs this
// library holds one copy of it (at its own address) until the process ends.
namespace cheb {
namespace {

constexpr size_t kScratchBytes = size_t(128) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

// device address of `scratch` on `dev`, looked up once per device with that
// device current (the array's name is a host-side stand-in, not an address)
int scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= 64) {
    set_error("device index out of range");
    return CHEB_ERR_DEVICE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = -1;
    int rc = hip_check(hipGetDevice(&cur), "hipGetDevice");
    if (rc) return rc;
    if (cur != dev && (rc = hip_check(hipSetDevice(dev), "hipSetDevice"))) return rc;
    void* ptr = nullptr;
    rc = hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (cur != dev) {
      const int rc2 = hip_check(hipSetDevice(cur), "hipSetDevice");
      if (!rc) rc = rc2;
    }
    if (rc) return rc;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return CHEB_OK;
}

}  // namespace
}  // namespace cheb

extern "C" int cheb_prolong_noalloc(const cheb_plan* coarse, const cheb_plan* fine, const void* u_c, void* u_f) {
  if (!coarse || !fine || !u_c || !u_f || u_c == u_f) {
    set_error("invalid argument");
    return CHEB_ERR_INVALID_ARG;
  }
  if (coarse->prec != fine->prec || coarse->device != fine->device) {
    set_error("coarse and fine plans must have the same precision and device");
    return CHEB_ERR_INVALID_ARG;
  }
  for (int a = 0; a < 3; ++a) {
    if (fine->g.n[a] < coarse->g.n[a]) {
      set_error("fine grid must not be smaller than the coarse grid");
      return CHEB_ERR_INVALID_ARG;
    }
    if (std::fabs(fine->g.lo[a] - coarse->g.lo[a]) > 0 || std::fabs(fine->g.hi[a] - coarse->g.hi[a]) > 0) {
      set_error("coarse and fine plans must describe the same box");
      return CHEB_ERR_INVALID_ARG;
    }
  }
  // intermediates after the z pass (nc0, nc1, nf2) and the y pass (nc0, nf1, nf2)
  const size_t esz = fine->prec == CHEB_F32 ? sizeof(float) : sizeof(double);
  const size_t nc0 = coarse->g.n[0], nc1 = coarse->g.n[1], nf1 = fine->g.n[1], nf2 = fine->g.n[2];
  const size_t b1 = round_up(nc0 * nc1 * nf2 * esz, 256);
  const size_t b2 = round_up(nc0 * nf1 * nf2 * esz, 256);
  if (b1 + b2 > kScratchBytes) {
    set_error("prolongation intermediates (" + std::to_string(b1 + b2) + " bytes) exceed the " +
              std::to_string(kScratchBytes) + "-byte static scratch of cheb_prolong_noalloc");
    return CHEB_ERR_WORKSPACE;
  }
  void* base = nullptr;
  int rc = scratch_address(fine->device, &base);
  if (rc) return rc;
  char* ws = (char*)base;
  if (fine->prec == CHEB_F32)
    return prolong_t<float>(coarse, fine, (const float*)u_c, (float*)u_f, (float*)ws, (float*)(ws + b1),
                            fine->stream);
  return prolong_t<double>(coarse, fine, (const double*)u_c, (double*)u_f, (double*)ws, (double*)(ws + b1),
                           fine->stream);
}
