// Device side of the LGMRES restart cycle (Algorithm 2's Krylov solver): the
// Hessenberg column of each Arnoldi step, its Givens rotations, the residual
// estimate and the convergence predicate, and the least-squares solve at the
// end of the cycle all run in single-wave kernels on the solver's stream, so
// the host enqueues Arnoldi steps without waiting for them.  The host reads
// the small head of the state once per step, one step behind the GPU, to know
// when a cycle has ended; it never sits between two steps.
//
// Each Gram-Schmidt pass is two launches: the multi-dot (k_gram_schmidt) and
// one workgroup that reduces its partial sums and forms the Hessenberg column
// (k_gs_column).
// The column update is the classical Gram-Schmidt of the multi-dot: with
// h_i = <v_i, w> and ||w||^2 from one pass, ||w - V h||^2 = ||w||^2 - ||h||^2;
// when that difference falls below kReorthEta2 ||w||^2 (severe cancellation,
// the Daniel-Gragg-Kaufman-Stewart test) the column is left open, the cycle
// pauses (`reorth` set, `active` cleared) and the host enqueues a second
// Gram-Schmidt pass for that column before it resumes.  Cancellation is rare,
// so a step normally costs the multi-dot, the column and one update.
#include <cmath>

#include "internal.h"

namespace cheb {

namespace {

constexpr int kW = 64;

__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ __launch_bounds__(kW) void k_arnoldi_init(ArnoldiState* st, double tol, double stall) {
  if (threadIdx.x == 0) {
    st->tol = tol;
    st->stall = stall;
    st->bprev = HUGE_VAL;
    st->active = 0;
    st->jend = 0;
    st->reorth = 0;
    st->breakdown = 0;
    st->stagnated = 0;
    st->direct = 0;
  }
}

// start of a restart cycle: dots[0] = ||r||^2 of the true residual r
__global__ __launch_bounds__(kW) void k_arnoldi_begin(ArnoldiState* st, const double* dots) {
  if (threadIdx.x != 0) return;
  const double b2 = dots[0];
  const double beta = std::sqrt(b2 > 0.0 ? b2 : 0.0);
  st->beta = beta;
  st->inv_beta = beta > 0.0 ? 1.0 / beta : 0.0;
  st->g[0] = beta;
  st->jend = 0;
  st->reorth = 0;
  st->direct = 0;
  st->breakdown = 0;
  st->est = beta;
  st->stagnated = (st->stall > 0.0 && beta > st->stall * st->bprev) ? 1 : 0;
  st->active = (beta > st->tol && std::isfinite(beta) && !st->stagnated) ? 1 : 0;
  st->bprev = beta;
}

// column j of the Hessenberg matrix from the multi-dot dots[0..j+1], in one
// wave (lane = 0..63; `col` is LDS scratch of 3 (kMaxKrylovCols + 2) entries)
// (pass 0: first Gram-Schmidt pass; pass 1: the re-orthogonalisation pass,
// whose coefficients add to the column), then -- unless pass 0 asks for
// re-orthogonalisation -- the Givens rotations, the residual estimate
// |g[j+1]| and the cycle's continuation flag.  The caller has checked that the
// pass runs (pass 0: the cycle is active; pass 1: re-orthogonalisation asked).
__device__ void arnoldi_column_wave(ArnoldiState* st, const double* dots, int j, int pass, int lane,
                                    double* col) {
  const int ld = kMaxKrylovCols;
  double* rc_ = col + (kMaxKrylovCols + 2);  // cs[i], sn[i] of the earlier columns, interleaved
  double ss = 0.0;
  for (int i = lane; i <= j; i += kW) {
    const double h = dots[i];
    ss = fma(h, h, ss);
    col[i] = pass == 0 ? h : st->H[i * ld + j] + h;
    if (i < j) {
      rc_[2 * i] = st->cs[i];
      rc_[2 * i + 1] = st->sn[i];
    }
  }
  ss = wave_sum64(ss);
  const double ww = dots[j + 1];
  const double hh2 = ww - ss;
  // the lanes' LDS writes of col before lane 0 reads them
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  if (pass == 0 && !(hh2 > kReorthEta2 * ww)) {
    // cancellation: keep the coefficients and pause the cycle; the host runs
    // the second pass for this column and resumes
    for (int i = lane; i <= j; i += kW) st->H[i * ld + j] = col[i];
    if (lane == 0) {
      st->reorth = 1;
      st->direct = 0;
      st->active = 0;
    }
    return;
  }
  const double hn = hh2 > 0.0 ? std::sqrt(hh2) : 0.0;
  if (lane == 0) {
    // previous rotations applied to the new column (in LDS)
    double a = col[0];
    for (int i = 0; i < j; ++i) {
      const double b = col[i + 1];
      const double c = rc_[2 * i], s = rc_[2 * i + 1];
      col[i] = c * a + s * b;
      a = -s * a + c * b;
    }
    col[j] = a;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  for (int i = lane; i < j; i += kW) st->H[i * ld + j] = col[i];
  if (lane != 0) return;
  st->reorth = 0;
  st->hn = hn;
  st->inv_hn = hn > 0.0 ? 1.0 / hn : 0.0;
  const double a = col[j];
  const double bb = hn;
  const double r = std::hypot(a, bb);
  double c = 1.0, s = 0.0;
  if (r != 0.0) {
    c = a / r;
    s = bb / r;
  }
  st->cs[j] = c;
  st->sn[j] = s;
  st->H[j * ld + j] = r;
  st->H[(j + 1) * ld + j] = 0.0;
  const double gj = st->g[j];
  st->g[j + 1] = -s * gj;
  st->g[j] = c * gj;
  st->jend = j + 1;
  const double est = std::fabs(-s * gj);
  st->est = est;
  st->breakdown = (!(bb > 1e-300) || !(r > 0.0)) ? 1 : 0;
  st->active = (est <= st->tol || st->breakdown) ? 0 : 1;
  // the update that follows forms v_{j+1} unless the cycle ends here
  st->direct = st->active;
}

// One Gram-Schmidt pass of Arnoldi step j in two launches: the multi-dot
// <v_i, w> (i < nv) and <w, w> over the blocks' chunks (k_gram_schmidt), then
// one workgroup that sums the blocks' partial results and forms the Hessenberg
// column (k_gs_column).  PASS 0 runs while the cycle is active; PASS 1
// (re-orthogonalisation) only when pass 0 asked for it, and first replaces w
// by w - V h0 with h0 the pass-0 coefficients.  Partial sums are stored
// column-major ([c][block]) so each column is summed from contiguous memory,
// always in the same order, so results are reproducible.
constexpr int kGsThreads = 256;
constexpr int kGsEPT = 8;
constexpr int kGsChunk = kGsThreads * kGsEPT;
constexpr int kColThreads = 1024;  // the column kernel: one wave per column of partial sums (j < 16 in one round)

template <typename T, int PASS>
__global__ __launch_bounds__(kGsThreads) void k_gram_schmidt(const T* __restrict__ V, size_t ld, int nv, T* w,
                                                             size_t npts, const double* __restrict__ h0,
                                                             double* __restrict__ partials,
                                                             const ArnoldiState* st) {
  __shared__ double red[kGsThreads / 64][kMaxKrylovCols + 2];
  __shared__ double hs[kMaxKrylovCols + 2];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  if (PASS == 0 ? !st->active : !st->reorth) return;
  const int nb = gridDim.x;
  const size_t b0 = (size_t)blockIdx.x * kGsChunk;
  double wv[kGsEPT];
  size_t ix[kGsEPT];
#pragma unroll
  for (int e = 0; e < kGsEPT; ++e) {
    const size_t i = b0 + tid + (size_t)e * kGsThreads;
    ix[e] = i < npts ? i : npts - 1;
    wv[e] = i < npts ? double(w[i]) : 0.0;
  }
  if (PASS == 1) {
    for (int v = tid; v < nv; v += kGsThreads) hs[v] = h0[v];
    __syncthreads();
    for (int v = 0; v < nv; ++v) {
      const double hv = hs[v];
#pragma unroll
      for (int e = 0; e < kGsEPT; ++e) wv[e] = fma(-hv, double(V[(size_t)v * ld + ix[e]]), wv[e]);
    }
#pragma unroll
    for (int e = 0; e < kGsEPT; ++e) {
      const size_t i = b0 + tid + (size_t)e * kGsThreads;
      if (i < npts) {
        w[i] = T(wv[e]);
        wv[e] = double(T(wv[e]));  // the dots see the stored (rounded) vector
      }
    }
  }
  // basis vectors four at a time, all their loads issued before the products
  // (slots past the last vector load w; every index is clamped into range)
  for (int v0 = 0; v0 <= nv; v0 += 4) {
    T x[4][kGsEPT];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const T* Vi = v0 + g < nv ? V + (size_t)(v0 + g) * ld : w;
#pragma unroll
      for (int e = 0; e < kGsEPT; ++e) x[g][e] = Vi[ix[e]];
    }
    double acc[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      acc[g] = 0.0;
      if (v0 + g < nv) {
#pragma unroll
        for (int e = 0; e < kGsEPT; ++e) acc[g] = fma(wv[e], double(x[g][e]), acc[g]);
      } else {
#pragma unroll
        for (int e = 0; e < kGsEPT; ++e) acc[g] = fma(wv[e], wv[e], acc[g]);
      }
    }
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const double t = wave_sum64(acc[g]);
      if (lane == 0 && v0 + g <= nv) red[wave][v0 + g] = t;
    }
  }
  __syncthreads();
  for (int v = tid; v <= nv; v += kGsThreads) {
    double sum = 0.0;
#pragma unroll
    for (int q = 0; q < kGsThreads / 64; ++q) sum += red[q][v];
    partials[(size_t)v * nb + blockIdx.x] = sum;
  }
}

// column sums of the nb blocks' partial results (wave q takes columns q,
// q + 4, ...; lanes stride the blocks), then the Hessenberg column
// The step's status record (the state's head) then goes to host_head (pinned
// host memory, or null), written by lane 0 of wave 0 after the column, so the
// host reads it once the step's event has completed, with no copy launch.
__device__ __forceinline__ void head_to_host(const ArnoldiState* st, ArnoldiHead* host_head) {
  static_assert(sizeof(ArnoldiHead) % sizeof(double) == 0, "head copied as doubles");
  const double* src = reinterpret_cast<const double*>(static_cast<const ArnoldiHead*>(st));
  double* dst = reinterpret_cast<double*>(host_head);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(ArnoldiHead) / sizeof(double)); ++i) dst[i] = src[i];
}

template <int PASS>
__global__ __launch_bounds__(kColThreads) void k_gs_column(const double* __restrict__ partials, int nb, int nv,
                                                          double* dots, ArnoldiState* st, int j,
                                                          ArnoldiHead* host_head) {
  __shared__ double hs[kMaxKrylovCols + 2];
  __shared__ double col[3 * (kMaxKrylovCols + 2)];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  if (PASS == 0 ? !st->active : !st->reorth) {
    if (host_head && tid == 0) head_to_host(st, host_head);
    return;
  }
  for (int c = wave; c <= nv; c += kColThreads / 64) {
    const double* pc = partials + (size_t)c * nb;
    double s4[4] = {0.0, 0.0, 0.0, 0.0};
    int r = lane;
    for (; r + 192 < nb; r += 256) {
#pragma unroll
      for (int q = 0; q < 4; ++q) s4[q] += pc[r + 64 * q];
    }
    for (; r < nb; r += 64) s4[0] += pc[r];
    double sum = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    sum = wave_sum64(sum);
    if (lane == 0) hs[c] = sum;
  }
  __syncthreads();
  for (int v = tid; v <= nv; v += kColThreads) dots[v] = hs[v];
  if (wave == 0) {
    arnoldi_column_wave(st, hs, j, PASS, lane, col);
    // lane 0 wrote the head's scalars; the other lanes' H writes are not in it
    if (host_head && lane == 0) head_to_host(st, host_head);
  }
}

// y = R^{-1} g over the columns the cycle built (back-substitution)
__global__ __launch_bounds__(kW) void k_arnoldi_solve(ArnoldiState* st) {
  const int lane = threadIdx.x;
  const int jend = st->jend;
  const int ld = kMaxKrylovCols;
  for (int i = jend - 1; i >= 0; --i) {
    double t = 0.0;
    for (int l = i + 1 + lane; l < jend; l += kW) t = fma(st->H[i * ld + l], st->y[l], t);
    t = wave_sum64(t);
    if (lane == 0) {
      const double d = st->H[i * ld + i];
      st->y[i] = d != 0.0 ? (st->g[i] - t) / d : 0.0;
    }
    __syncthreads();
  }
}

template <typename T>
__global__ void k_scale_by(T* v, const double* dscale, size_t npts) {
  const double a = *dscale;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < npts; i += (size_t)gridDim.x * blockDim.x)
    v[i] = T(a * double(v[i]));
}

inline int blocks_for(size_t n) {
  size_t g = (n + 1023) / 1024;
  if (g < 1) g = 1;
  if (g > 8192) g = 8192;
  return (int)g;
}

}  // namespace

int arnoldi_init(ArnoldiState* st, double tol, double stall, hipStream_t s) {
  hipLaunchKernelGGL(k_arnoldi_init, dim3(1), dim3(kW), 0, s, st, tol, stall);
  return hip_check(hipGetLastError(), "arnoldi_init");
}

int arnoldi_begin(ArnoldiState* st, const double* dots, hipStream_t s) {
  hipLaunchKernelGGL(k_arnoldi_begin, dim3(1), dim3(kW), 0, s, st, dots);
  return hip_check(hipGetLastError(), "arnoldi_begin");
}

template <typename T>
int gram_schmidt(const T* V, size_t ld, int j, T* w, size_t npts, const double* h0, double* partials,
                 double* dots, ArnoldiState* st, int pass, hipStream_t s, ArnoldiHead* host_head) {
  if (j < 0 || j >= kMaxKrylovCols || npts == 0) {
    set_error("Arnoldi column out of range");
    return CHEB_ERR_INVALID_ARG;
  }
  const int nb = (int)((npts + kGsChunk - 1) / kGsChunk);
  if (pass == 0) {
    hipLaunchKernelGGL((k_gram_schmidt<T, 0>), dim3(nb), dim3(kGsThreads), 0, s, V, ld, j + 1, w, npts, h0,
                       partials, st);
    hipLaunchKernelGGL(k_gs_column<0>, dim3(1), dim3(kColThreads), 0, s, partials, nb, j + 1, dots, st, j,
                       host_head);
  } else {
    hipLaunchKernelGGL((k_gram_schmidt<T, 1>), dim3(nb), dim3(kGsThreads), 0, s, V, ld, j + 1, w, npts, h0,
                       partials, st);
    hipLaunchKernelGGL(k_gs_column<1>, dim3(1), dim3(kColThreads), 0, s, partials, nb, j + 1, dots, st, j,
                       host_head);
  }
  return hip_check(hipGetLastError(), "gram_schmidt");
}

int arnoldi_solve(ArnoldiState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_arnoldi_solve, dim3(1), dim3(kW), 0, s, st);
  return hip_check(hipGetLastError(), "arnoldi_solve");
}

template <typename T>
int scale_by(T* v, const double* dscale, size_t npts, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_by<T>, dim3(blocks_for(npts)), dim3(256), 0, s, v, dscale, npts);
  return hip_check(hipGetLastError(), "scale_by");
}

template int gram_schmidt<double>(const double*, size_t, int, double*, size_t, const double*, double*, double*,
                                  ArnoldiState*, int, hipStream_t, ArnoldiHead*);
template int gram_schmidt<float>(const float*, size_t, int, float*, size_t, const double*, double*, double*,
                                 ArnoldiState*, int, hipStream_t, ArnoldiHead*);
template int scale_by<double>(double*, const double*, size_t, hipStream_t);
template int scale_by<float>(float*, const double*, size_t, hipStream_t);

}  // namespace cheb
