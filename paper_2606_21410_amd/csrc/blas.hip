// Streaming vector kernels for the Krylov solver: one-pass multi-dot (all
// Gram-Schmidt coefficients and ||w||^2 in one read of the basis, FP64
// accumulation, deterministic two-stage reduction), fused update-and-scale,
// linear combinations, precision casts and small pointwise kernels.
#include "internal.h"

namespace cheb {

namespace {

constexpr int kThreads = 256;
constexpr int kEPT = 8;                        // elements per thread in the multi-dot
constexpr int kChunk = kThreads * kEPT;        // elements per multi-dot block
constexpr int kMaxDots = 72;

inline int grid_for(size_t n, int per_block = kThreads * 4, int cap = 8192) {
  size_t g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > (size_t)cap) g = cap;
  return (int)g;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Basis vectors are taken kGroup at a time: their loads are all issued before
// the first product, so a block keeps kGroup * kEPT loads per thread in flight.
// The per-vector accumulation order is that of one vector at a time.  Slots of
// a group past the last vector load w (V may be null when nv is 0), and every
// index is clamped into [0, npts), so all loads stay inside w and the basis.
constexpr int kGroup = 4;

template <typename T>
__global__ __launch_bounds__(kThreads) void k_multidot(const T* __restrict__ V, size_t ld, int nv,
                                                       const T* __restrict__ w, size_t npts,
                                                       double* __restrict__ partials, const int* gate) {
  if (gate && !*gate) return;  // device-side predicate (the Arnoldi re-orthogonalisation pass)
  __shared__ double red[kThreads / 64][kMaxDots];
  const size_t b0 = (size_t)blockIdx.x * kChunk;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  double wv[kEPT];
  size_t ix[kEPT];  // element index, clamped into range (its w value is 0 past the end)
#pragma unroll
  for (int e = 0; e < kEPT; ++e) {
    const size_t i = b0 + tid + (size_t)e * kThreads;
    ix[e] = i < npts ? i : npts - 1;
    wv[e] = i < npts ? double(w[i]) : 0.0;
  }
  for (int v0 = 0; v0 <= nv; v0 += kGroup) {
    T x[kGroup][kEPT];
#pragma unroll
    for (int g = 0; g < kGroup; ++g) {
      const T* Vi = v0 + g < nv ? V + (size_t)(v0 + g) * ld : w;
#pragma unroll
      for (int e = 0; e < kEPT; ++e) x[g][e] = Vi[ix[e]];
    }
    double acc[kGroup];
#pragma unroll
    for (int g = 0; g < kGroup; ++g) {
      acc[g] = 0.0;
      if (v0 + g < nv) {
#pragma unroll
        for (int e = 0; e < kEPT; ++e) acc[g] = fma(wv[e], double(x[g][e]), acc[g]);
      } else {
#pragma unroll
        for (int e = 0; e < kEPT; ++e) acc[g] = fma(wv[e], wv[e], acc[g]);
      }
    }
#pragma unroll
    for (int g = 0; g < kGroup; ++g) {
      const double t = wave_sum(acc[g]);
      if (lane == 0 && v0 + g <= nv) red[wave][v0 + g] = t;
    }
  }
  __syncthreads();
  for (int v = tid; v <= nv; v += kThreads) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kThreads / 64; ++q) s += red[q][v];
    partials[(size_t)blockIdx.x * (nv + 1) + v] = s;
  }
}

__global__ __launch_bounds__(kThreads) void k_reduce_cols(const double* __restrict__ partials, int rows,
                                                         int cols, double* __restrict__ out,
                                                         const int* gate = nullptr) {
  if (gate && !*gate) return;
  __shared__ double red[kThreads / 64];
  const int c = blockIdx.x, tid = threadIdx.x;
  double s = 0.0;
  for (int r = tid; r < rows; r += kThreads) s += partials[(size_t)r * cols + c];
  s = wave_sum(s);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int q = 0; q < kThreads / 64; ++q) t += red[q];
    out[c] = t;
  }
}

// out = (w - sum_v h_v V_v) * scale; kUE elements per thread per step, with
// the basis loads of kGroup vectors issued together
constexpr int kUE = 4;

template <typename T>
__global__ __launch_bounds__(kThreads) void k_update_scale(const T* __restrict__ V, size_t ld, int nv,
                                                           const double* __restrict__ h, const T* w, T* out,
                                                           double scale, size_t npts, const double* dscale,
                                                           const int* gate) {
  if (gate && !*gate) return;
  if (dscale) scale = *dscale;
  __shared__ double hs[kMaxDots];
  for (int v = threadIdx.x; v < nv; v += kThreads) hs[v] = h[v];
  __syncthreads();
  const size_t step = (size_t)gridDim.x * kThreads * kUE;
  for (size_t i0 = (size_t)blockIdx.x * kThreads * kUE + threadIdx.x; i0 < npts; i0 += step) {
    size_t ix[kUE];
    double acc[kUE];
#pragma unroll
    for (int q = 0; q < kUE; ++q) {
      const size_t i = i0 + (size_t)q * kThreads;
      ix[q] = i < npts ? i : npts - 1;
      acc[q] = double(w[ix[q]]);
    }
    int v = 0;
    for (; v + kGroup <= nv; v += kGroup) {
      T x[kGroup][kUE];
#pragma unroll
      for (int g = 0; g < kGroup; ++g)
#pragma unroll
        for (int q = 0; q < kUE; ++q) x[g][q] = V[(size_t)(v + g) * ld + ix[q]];
#pragma unroll
      for (int g = 0; g < kGroup; ++g)
#pragma unroll
        for (int q = 0; q < kUE; ++q) acc[q] = fma(-hs[v + g], double(x[g][q]), acc[q]);
    }
    for (; v < nv; ++v)
#pragma unroll
      for (int q = 0; q < kUE; ++q) acc[q] = fma(-hs[v], double(V[(size_t)v * ld + ix[q]]), acc[q]);
#pragma unroll
    for (int q = 0; q < kUE; ++q)
      if (i0 + (size_t)q * kThreads < npts) out[i0 + (size_t)q * kThreads] = T(acc[q] * scale);
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_lincomb(const T* __restrict__ V, size_t ld, int nv,
                                                      const double* __restrict__ c, T* out, int accumulate,
                                                      size_t npts) {
  __shared__ double cs[kMaxDots];
  for (int v = threadIdx.x; v < nv; v += kThreads) cs[v] = c[v];
  __syncthreads();
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < npts; i += (size_t)gridDim.x * kThreads) {
    double acc = accumulate ? double(out[i]) : 0.0;
    for (int v = 0; v < nv; ++v) acc = fma(cs[v], double(V[(size_t)v * ld + i]), acc);
    out[i] = T(acc);
  }
}

template <typename T>
__global__ void k_axpby(T* y, const T* x, double alpha, double beta, size_t npts) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < npts; i += (size_t)gridDim.x * blockDim.x)
    y[i] = T(alpha * double(x[i]) + (beta == 0.0 ? 0.0 : beta * double(y[i])));
}

template <typename T>
__global__ void k_copy_scale(T* y, const T* x, double alpha, size_t npts) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < npts; i += (size_t)gridDim.x * blockDim.x)
    y[i] = T(alpha * double(x[i]));
}

__global__ void k_cast_f64_f32(float* y, const double* x, double alpha, size_t npts) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < npts; i += (size_t)gridDim.x * blockDim.x)
    y[i] = float(alpha * x[i]);
}

__global__ void k_add_f32_to_f64(double* y, const float* x, double alpha, size_t npts) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < npts; i += (size_t)gridDim.x * blockDim.x)
    y[i] = fma(alpha, double(x[i]), y[i]);
}

template <typename T>
__global__ void k_fill(T* y, double v, size_t npts) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < npts; i += (size_t)gridDim.x * blockDim.x)
    y[i] = T(v);
}

__device__ __forceinline__ bool is_interior(size_t i, int n0, int n1, int n2) {
  const int k = (int)(i % n2);
  const size_t t = i / n2;
  const int j = (int)(t % n1);
  const int ii = (int)(t / n1);
  return ii > 0 && ii < n0 - 1 && j > 0 && j < n1 - 1 && k > 0 && k < n2 - 1;
}

template <typename T>
__global__ void k_rhs_reduced(T* y, const T* f, int n0, int n1, int n2) {
  const size_t npts = (size_t)n0 * n1 * n2;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < npts; i += (size_t)gridDim.x * blockDim.x)
    y[i] = is_interior(i, n0, n1, n2) ? T(f[i] - y[i]) : T(0);
}

template <typename T>
__global__ void k_mask_interior(T* y, int n0, int n1, int n2) {
  const size_t npts = (size_t)n0 * n1 * n2;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < npts; i += (size_t)gridDim.x * blockDim.x)
    if (!is_interior(i, n0, n1, n2)) y[i] = T(0);
}

__global__ void k_picard_coeff(double* K, const double* K0, const double* u, size_t npts) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < npts; i += (size_t)gridDim.x * blockDim.x) {
    const double v = u[i];
    K[i] = K0[i] * (1.0 + 0.5 * v * v);
  }
}

// reciprocal law of the nonlinear example: k = K0 / (1 + alpha T) and
// k' = -alpha K0 / (1 + alpha T)^2 = -alpha k / (1 + alpha T)
__global__ void k_newton_coeff(double* k, double* kp, const double* K0, const double* T, double alpha,
                               size_t npts) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < npts; i += (size_t)gridDim.x * blockDim.x) {
    const double d = 1.0 + alpha * T[i];
    const double kv = K0[i] / d;
    k[i] = kv;
    kp[i] = -alpha * kv / d;
  }
}

__global__ void k_vmul(double* y, const double* a, const double* b, size_t npts) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < npts; i += (size_t)gridDim.x * blockDim.x)
    y[i] = a[i] * b[i];
}

__global__ void k_grad_acc(double* g, const double* du, const double* dl, int first, size_t npts) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < npts; i += (size_t)gridDim.x * blockDim.x)
    g[i] = (first ? 0.0 : g[i]) + du[i] * dl[i];
}

__global__ void k_grad_finish(double* g, const double* K, size_t npts) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < npts; i += (size_t)gridDim.x * blockDim.x)
    g[i] = -K[i] * g[i];
}

template <typename T>
__global__ void k_check_pos(const T* K, size_t npts, int* flag) {
  int bad = 0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < npts; i += (size_t)gridDim.x * blockDim.x) {
    const T v = K[i];
    if (!(v > T(0)) || !isfinite(v)) bad = 1;
  }
  if (bad) atomicOr(flag, 1);
}

__global__ __launch_bounds__(kThreads) void k_cc_dot(const double* a, const double* b, const double* wx,
                                                     const double* wy, const double* wz, int n0, int n1,
                                                     int n2, double* partials) {
  __shared__ double red[kThreads / 64];
  const size_t npts = (size_t)n0 * n1 * n2;
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < npts; i += (size_t)gridDim.x * kThreads) {
    const int k = (int)(i % n2);
    const size_t t = i / n2;
    const int j = (int)(t % n1);
    const int ii = (int)(t / n1);
    acc = fma(wx[ii] * wy[j] * wz[k], a[i] * b[i], acc);
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int q = 0; q < kThreads / 64; ++q) s += red[q];
    partials[blockIdx.x] = s;
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_vsum(const T* x, size_t npts, double* partials) {
  __shared__ double red[kThreads / 64];
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < npts; i += (size_t)gridDim.x * kThreads)
    acc += double(x[i]);
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int q = 0; q < kThreads / 64; ++q) s += red[q];
    partials[blockIdx.x] = s;
  }
}

}  // namespace

template <typename T>
int vsum(const T* x, size_t npts, double* partials, double* out, hipStream_t s) {
  const int blocks = grid_for(npts, kThreads * 4, 1024);
  hipLaunchKernelGGL(k_vsum<T>, dim3(blocks), dim3(kThreads), 0, s, x, npts, partials);
  hipLaunchKernelGGL(k_reduce_cols, dim3(1), dim3(kThreads), 0, s, partials, blocks, 1, out);
  return hip_check(hipGetLastError(), "vsum");
}
template int vsum<double>(const double*, size_t, double*, double*, hipStream_t);
template int vsum<float>(const float*, size_t, double*, double*, hipStream_t);

size_t multidot_partials_len(size_t npts, int nv) {
  const size_t blocks = (npts + kChunk - 1) / kChunk;
  return (blocks < 1 ? 1 : blocks) * (size_t)(nv + 1) + 4096;
}

template <typename T>
int multidot(const T* V, size_t ld, int nv, const T* w, size_t npts, double* partials, double* out,
             hipStream_t s, const int* gate) {
  if (nv + 1 > kMaxDots) {
    set_error("too many vectors in multi-dot");
    return CHEB_ERR_INVALID_ARG;
  }
  if (npts == 0) {  // every dot product is empty: zero rows reduce to 0
    hipLaunchKernelGGL(k_reduce_cols, dim3(nv + 1), dim3(kThreads), 0, s, partials, 0, nv + 1, out, gate);
    return hip_check(hipGetLastError(), "multidot");
  }
  const int blocks = (int)((npts + kChunk - 1) / kChunk);
  hipLaunchKernelGGL(k_multidot<T>, dim3(blocks), dim3(kThreads), 0, s, V, ld, nv, w, npts, partials, gate);
  hipLaunchKernelGGL(k_reduce_cols, dim3(nv + 1), dim3(kThreads), 0, s, partials, blocks, nv + 1, out, gate);
  return hip_check(hipGetLastError(), "multidot");
}

template <typename T>
int update_scale(const T* V, size_t ld, int nv, const double* h, const T* w, T* out, double scale,
                 size_t npts, hipStream_t s, const double* dscale, const int* gate) {
  if (nv > kMaxDots) {
    set_error("too many vectors in update");
    return CHEB_ERR_INVALID_ARG;
  }
  hipLaunchKernelGGL(k_update_scale<T>, dim3(grid_for(npts)), dim3(kThreads), 0, s, V, ld, nv, h, w, out,
                     scale, npts, dscale, gate);
  return hip_check(hipGetLastError(), "update_scale");
}

template <typename T>
int lincomb(const T* V, size_t ld, int nv, const double* c, T* out, int accumulate, size_t npts,
            hipStream_t s) {
  if (nv > kMaxDots) {
    set_error("too many vectors in combination");
    return CHEB_ERR_INVALID_ARG;
  }
  hipLaunchKernelGGL(k_lincomb<T>, dim3(grid_for(npts)), dim3(kThreads), 0, s, V, ld, nv, c, out,
                     accumulate, npts);
  return hip_check(hipGetLastError(), "lincomb");
}

template <typename T>
int axpby(T* y, const T* x, double alpha, double beta, size_t npts, hipStream_t s) {
  hipLaunchKernelGGL(k_axpby<T>, dim3(grid_for(npts)), dim3(kThreads), 0, s, y, x, alpha, beta, npts);
  return hip_check(hipGetLastError(), "axpby");
}

template <typename T>
int copy_scale(T* y, const T* x, double alpha, size_t npts, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_scale<T>, dim3(grid_for(npts)), dim3(kThreads), 0, s, y, x, alpha, npts);
  return hip_check(hipGetLastError(), "copy_scale");
}

int cast_f64_f32(float* y, const double* x, double alpha, size_t npts, hipStream_t s) {
  hipLaunchKernelGGL(k_cast_f64_f32, dim3(grid_for(npts)), dim3(kThreads), 0, s, y, x, alpha, npts);
  return hip_check(hipGetLastError(), "cast");
}

int add_f32_to_f64(double* y, const float* x, double alpha, size_t npts, hipStream_t s) {
  hipLaunchKernelGGL(k_add_f32_to_f64, dim3(grid_for(npts)), dim3(kThreads), 0, s, y, x, alpha, npts);
  return hip_check(hipGetLastError(), "add_f32_to_f64");
}

template <typename T>
int fill(T* y, double v, size_t npts, hipStream_t s) {
  hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(npts)), dim3(kThreads), 0, s, y, v, npts);
  return hip_check(hipGetLastError(), "fill");
}

template <typename T>
int rhs_reduced(T* y, const T* f, const int* n, hipStream_t s) {
  const size_t npts = (size_t)n[0] * n[1] * n[2];
  hipLaunchKernelGGL(k_rhs_reduced<T>, dim3(grid_for(npts)), dim3(kThreads), 0, s, y, f, n[0], n[1], n[2]);
  return hip_check(hipGetLastError(), "rhs_reduced");
}

template <typename T>
int mask_interior(T* y, const int* n, hipStream_t s) {
  const size_t npts = (size_t)n[0] * n[1] * n[2];
  hipLaunchKernelGGL(k_mask_interior<T>, dim3(grid_for(npts)), dim3(kThreads), 0, s, y, n[0], n[1], n[2]);
  return hip_check(hipGetLastError(), "mask_interior");
}

int picard_coeff(double* K, const double* K0, const double* u, size_t npts, hipStream_t s) {
  hipLaunchKernelGGL(k_picard_coeff, dim3(grid_for(npts)), dim3(kThreads), 0, s, K, K0, u, npts);
  return hip_check(hipGetLastError(), "picard_coeff");
}

int newton_coeff(double* k, double* kp, const double* K0, const double* T, double alpha, size_t npts,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_newton_coeff, dim3(grid_for(npts)), dim3(kThreads), 0, s, k, kp, K0, T, alpha, npts);
  return hip_check(hipGetLastError(), "newton_coeff");
}

int vmul(double* y, const double* a, const double* b, size_t npts, hipStream_t s) {
  hipLaunchKernelGGL(k_vmul, dim3(grid_for(npts)), dim3(kThreads), 0, s, y, a, b, npts);
  return hip_check(hipGetLastError(), "vmul");
}

int grad_accumulate(double* g, const double* du, const double* dl, int first, size_t npts, hipStream_t s) {
  hipLaunchKernelGGL(k_grad_acc, dim3(grid_for(npts)), dim3(kThreads), 0, s, g, du, dl, first, npts);
  return hip_check(hipGetLastError(), "grad_accumulate");
}

int grad_finish(double* g, const double* K, size_t npts, hipStream_t s) {
  hipLaunchKernelGGL(k_grad_finish, dim3(grid_for(npts)), dim3(kThreads), 0, s, g, K, npts);
  return hip_check(hipGetLastError(), "grad_finish");
}

int check_positive_finite(const double* K, size_t npts, int* dflag, hipStream_t s) {
  hipLaunchKernelGGL(k_check_pos<double>, dim3(grid_for(npts)), dim3(kThreads), 0, s, K, npts, dflag);
  return hip_check(hipGetLastError(), "check_positive");
}

int check_positive_finite_f32(const float* K, size_t npts, int* dflag, hipStream_t s) {
  hipLaunchKernelGGL(k_check_pos<float>, dim3(grid_for(npts)), dim3(kThreads), 0, s, K, npts, dflag);
  return hip_check(hipGetLastError(), "check_positive");
}

int cc_dot(const double* a, const double* b, const double* wx, const double* wy, const double* wz,
           const int* n, double* partials, double* out, hipStream_t s) {
  const size_t npts = (size_t)n[0] * n[1] * n[2];
  const int blocks = grid_for(npts, kThreads * 4, 1024);
  hipLaunchKernelGGL(k_cc_dot, dim3(blocks), dim3(kThreads), 0, s, a, b, wx, wy, wz, n[0], n[1], n[2],
                     partials);
  hipLaunchKernelGGL(k_reduce_cols, dim3(1), dim3(kThreads), 0, s, partials, blocks, 1, out);
  return hip_check(hipGetLastError(), "cc_dot");
}

#define CHEB_INST(T)                                                                                  \
  template int multidot<T>(const T*, size_t, int, const T*, size_t, double*, double*, hipStream_t,    \
                           const int*);                                                               \
  template int update_scale<T>(const T*, size_t, int, const double*, const T*, T*, double, size_t,    \
                               hipStream_t, const double*, const int*);                               \
  template int lincomb<T>(const T*, size_t, int, const double*, T*, int, size_t, hipStream_t);        \
  template int axpby<T>(T*, const T*, double, double, size_t, hipStream_t);                           \
  template int copy_scale<T>(T*, const T*, double, size_t, hipStream_t);                              \
  template int fill<T>(T*, double, size_t, hipStream_t);                                              \
  template int rhs_reduced<T>(T*, const T*, const int*, hipStream_t);                                 \
  template int mask_interior<T>(T*, const int*, hipStream_t);
CHEB_INST(double)
CHEB_INST(float)
#undef CHEB_INST

}  // namespace cheb

namespace cheb {
namespace {

// Stream copy with 16-byte accesses: the attainable-bandwidth reference the
// operator's HBM roofline fraction is quoted against.
// One 16-byte element per thread and one workgroup per 4 KiB: every wave
// issues its load at launch, with no loop-carried address arithmetic.
__global__ __launch_bounds__(256) void k_stream_copy(const double2* __restrict__ src, double2* __restrict__ dst,
                                                     size_t n2) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n2) dst[i] = src[i];
}

__global__ void k_copy_tail(const double* src, double* dst, size_t from, size_t n) {
  const size_t i = from + (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

}  // namespace
}  // namespace cheb

extern "C" int cheb_debug_copy(const void* src, void* dst, size_t n, void* stream) {
  using namespace cheb;
  if (!src || !dst) {
    set_error("null argument");
    return CHEB_ERR_INVALID_ARG;
  }
  if (((uintptr_t)src | (uintptr_t)dst) & 15) {
    set_error("cheb_debug_copy needs 16-byte aligned buffers");
    return CHEB_ERR_INVALID_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  const size_t n2 = n / 2;
  if (n2) {
    const size_t blocks = (n2 + 255) / 256;
    if (blocks > 0x7fffffffULL) {
      set_error("cheb_debug_copy: too many elements for one launch");
      return CHEB_ERR_INVALID_ARG;
    }
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, s, (const double2*)src, (double2*)dst,
                       n2);
  }
  if (n & 1) hipLaunchKernelGGL(k_copy_tail, dim3(1), dim3(64), 0, s, (const double*)src, (double*)dst, 2 * n2, n);
  return hip_check(hipGetLastError(), "cheb_debug_copy");
}
