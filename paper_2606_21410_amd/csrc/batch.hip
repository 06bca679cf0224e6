// Batched solver: many independent systems (for example the microstructures
// and load cases of a homogenisation study) solved in lockstep.  Every step of
// the Krylov method is a handful of launches for the whole batch: one
// matrix-core operator pass per size group and axis over a queue of tiles that
// spans all systems of the group, one fast-diagonalisation contraction per
// group of identical factors, and segmented vector kernels whose blocks each
// work on a chunk of one system.  Hessenberg matrices, Givens rotations and
// convergence decisions stay per system on the host (FP64); systems that have
// converged drop out of the tile queues.
//
// LGMRES is the restarted GMRES augmented with the previous corrections
// (Baker, Jessup & Manteuffel 2005; Section 2.3 uses it as the Krylov solver);
// the mixed-precision variant is FP64 iterative refinement around FP32 inner
// solves.  Fields of all systems are packed back to back (256-byte aligned)
// in caller-provided workspace.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "dense_pass.h"
#include "internal.h"

namespace cheb {
namespace {

constexpr int kChunk = 8192;  // elements per block of the segmented vector kernels
constexpr int kBT = 256;
constexpr int kMaxCoef = 80;  // per-system coefficient slots (m + k + 2 <= 72)
constexpr int kSide = 3;      // side streams the preconditioner groups run on

struct ApplyGroup {
  int rep;                    // system whose plan supplies N, box and tables
  bool dense;                 // matrix-core route (else per-system FFT passes)
  int shape[2] = {-1, -1};    // tile shape the autotuner chose, [FP64, FP32] (-1: not yet tuned)
  float tuned_us[2][2] = {{-1.f, -1.f}, {-1.f, -1.f}};  // its timings per shape
  std::vector<int> members;   // system ids
  DenseSys* dsys = nullptr;   // device table, one entry per member
  std::vector<DenseSys> htab; // its host copy
  int* dact = nullptr;        // device list of active member indices
  std::vector<int> hact;      // host copy of the active list last uploaded
};

struct PrecGroup {
  int rep;
  std::vector<int> members;
  size_t pack_off = 0;         // its region of the packed preconditioner scratch
  long long* doffs = nullptr;  // device: packed offsets of the active members
  int* dsys = nullptr;         // device: their system ids
  std::vector<int> hact;
};

}  // namespace
}  // namespace cheb

struct cheb_batch {
  int nprob;
  int prec;
  hipStream_t stream;
  std::vector<cheb_plan*> plans;
  std::vector<size_t> off, npts;
  // offset of each system's conductivity in the packed K: its own field's
  // offset, or that of the first system given the same K pointer and grid
  // size, which then holds the one packed copy (set per solve)
  std::vector<size_t> koff;
  size_t P;  // packed length in elements
  std::vector<cheb::ApplyGroup> groups;
  std::vector<cheb::PrecGroup> pgroups;
  // segmented-kernel chunk table (device)
  int nchunks;
  int* ch_sys;
  long long* ch_beg;
  int* ch_len;
  int* sys_c0;
  int* sys_nc;
  int* chl;       // device list of the chunks of the active systems
  int nchl;       // its length
  std::vector<int> hchl;
  std::vector<int> sys_c0_h, sys_nc_h;
  double* dcoef;  // nprob x kMaxCoef per-system coefficients
  double* dscal;  // nprob x 8 per-system scalars
  double* dkc;    // nprob mean conductivities
  int* dflag;
  double* hpin;   // pinned host staging: nprob x (kMaxCoef + 8) x 2 doubles
  void* ws;
  size_t ws_bytes;
  // the preconditioner groups are independent: they run on side streams
  // (default priority) forked from and joined to `stream` by events, so one
  // group's small contractions fill the dispatch gaps of another's
  hipStream_t side[cheb::kSide];
  hipEvent_t ev_fork, ev_join[cheb::kSide];
  int side_ok;
};

namespace cheb {
namespace {

// ---------------------------------------------------------------------------
// segmented vector kernels: block b works on chunk b of system ch_sys[b]
// ---------------------------------------------------------------------------
template <int G>
__device__ __forceinline__ void block_sum(double (&v)[G], double* red) {
#pragma unroll
  for (int t = 0; t < G; ++t) {
    double x = v[t];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    v[t] = x;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int t = 0; t < G; ++t) red[wv * G + t] = v[t];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int t = 0; t < G; ++t) v[t] = red[t] + red[G + t] + red[2 * G + t] + red[3 * G + t];
}

// partials[chunk][i] = <V_i, w> over the chunk for i < nv, <w, w> for i = nv;
// blockIdx.y selects the group of 8 outputs
template <typename T>
__global__ __launch_bounds__(kBT) void k_bdot(const T* __restrict__ V, size_t ld, int nv, const T* __restrict__ w,
                                              const int* __restrict__ chl, const long long* __restrict__ beg,
                                              const int* __restrict__ len, double* __restrict__ partials) {
  __shared__ double red[4 * 8];
  const int ch = chl[blockIdx.x], i0 = blockIdx.y * 8, nv1 = nv + 1;
  const long long b = beg[ch];
  const int L = len[ch];
  double acc[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) acc[t] = 0.0;
  for (int e = threadIdx.x; e < L; e += kBT) {
    const double wv = double(w[b + e]);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int i = i0 + t;
      if (i < nv) acc[t] += double(V[(size_t)i * ld + b + e]) * wv;
      else if (i == nv) acc[t] += wv * wv;
    }
  }
  block_sum<8>(acc, red);
  if (threadIdx.x == 0)
#pragma unroll
    for (int t = 0; t < 8; ++t)
      if (i0 + t < nv1) partials[(size_t)ch * nv1 + i0 + t] = acc[t];
}

// out[s][i] = sum over the chunks of system s
__global__ __launch_bounds__(kBT) void k_breduce(const double* __restrict__ partials, int nv1,
                                                 const int* __restrict__ c0, const int* __restrict__ nc,
                                                 double* __restrict__ out, int ostride) {
  const int s = blockIdx.x;
  for (int i = threadIdx.x; i < nv1; i += kBT) {
    double t = 0.0;
    for (int c = 0; c < nc[s]; ++c) t += partials[(size_t)(c0[s] + c) * nv1 + i];
    out[(size_t)s * ostride + i] = t;
  }
}

// out = (w - sum_i h[s][i] V_i) * scale[s]   (out may alias w)
template <typename T>
__global__ __launch_bounds__(kBT) void k_bupdate(const T* __restrict__ V, size_t ld, int nv, const double* h,
                                                 int hstride, const double* scale, int sstride, const T* w, T* out,
                                                 const int* __restrict__ chl, const int* __restrict__ sysv,
                                                 const long long* __restrict__ beg, const int* __restrict__ len) {
  const int ch = chl[blockIdx.x], s = sysv[ch];
  const long long b = beg[ch];
  const int L = len[ch];
  const double* hs = h + (size_t)s * hstride;
  const double sc = scale[(size_t)s * sstride];
  for (int e = threadIdx.x; e < L; e += kBT) {
    double x = double(w[b + e]);
    for (int i = 0; i < nv; ++i) x -= hs[i] * double(V[(size_t)i * ld + b + e]);
    out[b + e] = T(x * sc);
  }
}

// out (+)= sum_i c[s][i] V_i; terms with a zero coefficient are skipped, so
// basis columns a system never wrote (it stopped early) are never read
template <typename T>
__global__ __launch_bounds__(kBT) void k_blincomb(const T* __restrict__ V, size_t ld, int nv, const double* c,
                                                  int cstride, T* out, int accumulate, const int* __restrict__ chl,
                                                  const int* __restrict__ sysv, const long long* __restrict__ beg,
                                                  const int* __restrict__ len) {
  const int ch = chl[blockIdx.x], s = sysv[ch];
  const long long b = beg[ch];
  const int L = len[ch];
  const double* cs = c + (size_t)s * cstride;
  for (int e = threadIdx.x; e < L; e += kBT) {
    double x = accumulate ? double(out[b + e]) : 0.0;
    for (int i = 0; i < nv; ++i)
      if (cs[i] != 0.0) x += cs[i] * double(V[(size_t)i * ld + b + e]);
    out[b + e] = T(x);
  }
}

// y = alpha[s] x + beta[s] y   (alpha at scal[s*stride + ia], beta at + ib)
template <typename TY, typename TX>
__global__ __launch_bounds__(kBT) void k_baxpby(TY* y, const TX* __restrict__ x, const double* scal, int stride,
                                                int ia, int ib, const int* __restrict__ chl,
                                                const int* __restrict__ sysv, const long long* __restrict__ beg,
                                                const int* __restrict__ len) {
  const int ch = chl[blockIdx.x], s = sysv[ch];
  const long long b = beg[ch];
  const int L = len[ch];
  const double al = scal[(size_t)s * stride + ia];
  const double be = ib >= 0 ? scal[(size_t)s * stride + ib] : 0.0;
  for (int e = threadIdx.x; e < L; e += kBT) {
    const double yv = ib >= 0 ? double(y[b + e]) : 0.0;
    y[b + e] = TY(al * double(x[b + e]) + be * yv);
  }
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------
struct Carve {
  char* base;
  size_t off;
  template <typename U>
  U* take(size_t count) {
    U* p = base ? reinterpret_cast<U*>(base + off) : nullptr;
    off += round_up(count * sizeof(U), 256);
    return p;
  }
};

template <typename T>
struct BKrylov {
  T *V, *Z, *w, *wp, *pa, *pb;
  size_t ld;
  int m, k;
};

struct BScratch {
  double* partials;
  double* dots;  // nprob x kMaxCoef
};

struct BParams {
  double rtol = 1e-10, atol = 0.0;
  int maxiter = 10000, m = 30, k = 3;
  double ir_rtol = 1e-3;
  int ir_max = 50;
  bool warm = false, precond = false;
};

BParams bparams(const cheb_solve_opts* o) {
  BParams p;
  if (!o) return p;
  if (o->rtol > 0) p.rtol = o->rtol;
  if (o->atol > 0) p.atol = o->atol;
  if (o->maxiter > 0) p.maxiter = o->maxiter;
  if (o->inner_m > 0) p.m = o->inner_m;
  p.k = o->outer_k == 0 ? 3 : (o->outer_k < 0 ? 0 : o->outer_k);
  if (o->ir_inner_rtol > 0) p.ir_rtol = o->ir_inner_rtol;
  if (o->ir_max_outer > 0) p.ir_max = o->ir_max_outer;
  p.warm = (o->flags & 1) != 0;
  p.precond = (o->flags & 2) != 0;
  return p;
}

template <typename T>
void carve_bkrylov(Carve& c, size_t P, const BParams& bp, BKrylov<T>& kw) {
  kw.ld = round_up(P, 64);
  kw.m = bp.m;
  kw.k = bp.k;
  kw.V = c.take<T>(kw.ld * (bp.m + bp.k + 1));  // Arnoldi basis of the augmented space
  kw.Z = c.take<T>(kw.ld * (bp.k > 0 ? bp.k : 1));
  kw.w = c.take<T>(kw.ld);
  kw.wp = c.take<T>(kw.ld);
  kw.pa = bp.precond ? c.take<T>(kw.ld) : nullptr;
  kw.pb = bp.precond ? c.take<T>(kw.ld) : nullptr;
}

struct BWS {
  double *K64, *bt, *x, *r, *t1;
  float *K32, *b32, *d32;
  BKrylov<double> kw64;
  BKrylov<float> kw32;
  BScratch sc;
};

size_t carve_batch(cheb_batch* B, const BParams& bp, char* base, BWS& w) {
  Carve c{base, 0};
  const size_t P = round_up(B->P, 64);
  w.K64 = c.take<double>(P);
  w.bt = c.take<double>(P);
  w.x = c.take<double>(P);
  w.r = c.take<double>(P);
  w.t1 = c.take<double>(P);
  w.K32 = w.b32 = w.d32 = nullptr;
  if (B->prec == CHEB_MIXED) {
    w.K32 = c.take<float>(P);
    w.b32 = c.take<float>(P);
    w.d32 = c.take<float>(P);
    carve_bkrylov<float>(c, B->P, bp, w.kw32);
  } else {
    carve_bkrylov<double>(c, B->P, bp, w.kw64);
  }
  w.sc.partials = c.take<double>((size_t)B->nchunks * (bp.m + bp.k + 2) + 1024);
  w.sc.dots = c.take<double>((size_t)B->nprob * kMaxCoef);
  return c.off;
}

int bsync(cheb_batch* B) { return hip_check(hipStreamSynchronize(B->stream), "hipStreamSynchronize"); }

// per-system scalars: host staging -> device (async; the staging buffer is
// reused only after the next synchronising readback)
int upload(cheb_batch* B, double* dev, const double* host_src, size_t count, int half) {
  double* hp = B->hpin + (size_t)half * B->nprob * (kMaxCoef + 8);
  std::memcpy(hp, host_src, count * sizeof(double));
  return hip_check(hipMemcpyAsync(dev, hp, count * sizeof(double), hipMemcpyHostToDevice, B->stream),
                   "hipMemcpyAsync(H2D)");
}

template <typename T>
int bdots(cheb_batch* B, const T* V, size_t ld, int nv, const T* w, BScratch& sc, std::vector<double>& out) {
  const int nv1 = nv + 1;
  if (B->nchl == 0) {
    out.assign((size_t)B->nprob * kMaxCoef, 0.0);
    return CHEB_OK;
  }
  dim3 grid(B->nchl, (nv1 + 7) / 8);
  hipLaunchKernelGGL(k_bdot<T>, grid, dim3(kBT), 0, B->stream, V, ld, nv, w, B->chl, B->ch_beg, B->ch_len,
                     sc.partials);
  int rc = hip_check(hipGetLastError(), "batched multi-dot");
  if (rc) return rc;
  hipLaunchKernelGGL(k_breduce, dim3(B->nprob), dim3(kBT), 0, B->stream, sc.partials, nv1, B->sys_c0, B->sys_nc,
                     sc.dots, kMaxCoef);
  rc = hip_check(hipGetLastError(), "batched reduce");
  if (rc) return rc;
  double* hp = B->hpin + (size_t)2 * B->nprob * (kMaxCoef + 8);
  rc = hip_check(hipMemcpyAsync(hp, sc.dots, (size_t)B->nprob * kMaxCoef * sizeof(double), hipMemcpyDeviceToHost,
                                B->stream),
                 "hipMemcpyAsync(D2H)");
  if (!rc) rc = bsync(B);
  if (rc) return rc;
  out.assign(hp, hp + (size_t)B->nprob * kMaxCoef);
  return CHEB_OK;
}

template <typename T>
int bupdate(cheb_batch* B, const T* V, size_t ld, int nv, const T* w, T* out) {
  if (B->nchl == 0) return CHEB_OK;
  hipLaunchKernelGGL(k_bupdate<T>, dim3(B->nchl), dim3(kBT), 0, B->stream, V, ld, nv, B->dcoef, kMaxCoef,
                     B->dscal, 8, w, out, B->chl, B->ch_sys, B->ch_beg, B->ch_len);
  return hip_check(hipGetLastError(), "batched update");
}

template <typename T>
int blincomb(cheb_batch* B, const T* V, size_t ld, int nv, int coef_off, T* out, int acc) {
  if (B->nchl == 0) return CHEB_OK;
  hipLaunchKernelGGL(k_blincomb<T>, dim3(B->nchl), dim3(kBT), 0, B->stream, V, ld, nv, B->dcoef + coef_off,
                     kMaxCoef, out, acc, B->chl, B->ch_sys, B->ch_beg, B->ch_len);
  return hip_check(hipGetLastError(), "batched linear combination");
}

template <typename TY, typename TX>
int baxpby(cheb_batch* B, TY* y, const TX* x, int ia, int ib) {
  if (B->nchl == 0) return CHEB_OK;
  hipLaunchKernelGGL((k_baxpby<TY, TX>), dim3(B->nchl), dim3(kBT), 0, B->stream, y, x, B->dscal, 8, ia, ib,
                     B->chl, B->ch_sys, B->ch_beg, B->ch_len);
  return hip_check(hipGetLastError(), "batched axpby");
}

// active lists of the apply groups, preconditioner groups and vector kernels
// for the systems flagged in `on`
int set_active(cheb_batch* B, const std::vector<char>& on) {
  {
    std::vector<int> c;
    for (int s = 0; s < B->nprob; ++s)
      if (on[s])
        for (int k = 0; k < B->sys_nc_h[s]; ++k) c.push_back(B->sys_c0_h[s] + k);
    if (c != B->hchl) {
      if (!c.empty()) {
        int rc = hip_check(hipMemcpyAsync(B->chl, c.data(), c.size() * sizeof(int), hipMemcpyHostToDevice, B->stream),
                           "hipMemcpyAsync(chunk list)");
        if (!rc) rc = bsync(B);
        if (rc) return rc;
      }
      B->hchl = c;
      B->nchl = (int)c.size();
    }
  }
  for (auto& g : B->groups) {
    std::vector<int> a;
    for (int k = 0; k < (int)g.members.size(); ++k)
      if (on[g.members[k]]) a.push_back(k);
    if (a != g.hact && g.dense && !a.empty()) {
      int rc = hip_check(hipMemcpyAsync(g.dact, a.data(), a.size() * sizeof(int), hipMemcpyHostToDevice, B->stream),
                         "hipMemcpyAsync(active list)");
      if (rc) return rc;
      // the list lives in pageable memory: wait for the copy before it changes
      rc = bsync(B);
      if (rc) return rc;
    }
    g.hact = a;
  }
  for (auto& g : B->pgroups) {
    std::vector<int> a;
    for (int s : g.members)
      if (on[s]) a.push_back(s);
    if (a != g.hact && !a.empty()) {
      std::vector<long long> offs(a.size());
      for (size_t k = 0; k < a.size(); ++k) offs[k] = (long long)B->off[a[k]];
      int rc = hip_check(hipMemcpyAsync(g.doffs, offs.data(), offs.size() * sizeof(long long), hipMemcpyHostToDevice,
                                        B->stream),
                         "hipMemcpyAsync(preconditioner members)");
      if (!rc)
        rc = hip_check(hipMemcpyAsync(g.dsys, a.data(), a.size() * sizeof(int), hipMemcpyHostToDevice, B->stream),
                       "hipMemcpyAsync(preconditioner members)");
      if (!rc) rc = bsync(B);
      if (rc) return rc;
    }
    g.hact = a;
  }
  return CHEB_OK;
}

// fork: the side streams wait for the work enqueued so far on the batch's
// stream; join: the batch's stream waits for what the first `used` side
// streams were given
int side_fork(cheb_batch* B) {
  int rc = hip_check(hipEventRecord(B->ev_fork, B->stream), "hipEventRecord");
  for (int k = 0; k < kSide && !rc; ++k) rc = hip_check(hipStreamWaitEvent(B->side[k], B->ev_fork, 0), "hipStreamWaitEvent");
  return rc;
}
int side_join(cheb_batch* B, int used) {
  int rc = CHEB_OK;
  for (int k = 0; k < kSide && k < used && !rc; ++k) {
    rc = hip_check(hipEventRecord(B->ev_join[k], B->side[k]), "hipEventRecord");
    if (!rc) rc = hip_check(hipStreamWaitEvent(B->stream, B->ev_join[k], 0), "hipStreamWaitEvent");
  }
  return rc;
}

// y = A x for the active systems (reduced operator, packed fields); the
// groups are independent and run on the side streams
template <typename T>
int bapply(cheb_batch* B, const T* K, const T* x, T* y) {
  int nact = 0;
  for (auto& g : B->groups) nact += g.hact.empty() ? 0 : 1;
  const bool fork = B->side_ok && nact > 1;
  int rc = fork ? side_fork(B) : CHEB_OK;
  if (rc) return rc;
  int i = 0;
  for (auto& g : B->groups) {
    if (rc) break;
    if (g.hact.empty()) continue;
    hipStream_t st = fork ? B->side[i % kSide] : B->stream;
    ++i;
    const cheb_plan* rep = B->plans[g.rep];
    if (g.dense) {
      for (int pass = 0; pass < 3 && !rc; ++pass) {
        const int axis = 2 - pass;
        rc = launch_dense_batch<T>(rep, axis, pass == 0, K, x, y, g.dsys, g.dact, (int)g.hact.size(), st);
      }
    } else {
      for (int k : g.hact) {
        const int s = g.members[k];
        const size_t o = B->off[s];
        rc = apply_t<T>(B->plans[s], K + B->koff[s], x + o, y + o, 1, st);
        if (rc) break;
      }
    }
  }
  // joined also after an error, so nothing enqueued here outlives the call's stream order
  if (fork) {
    const int rj = side_join(B, i);
    if (!rc) rc = rj;
  }
  return rc;
}

// each group packs its members' interiors into its own region of pa / pb, so
// the groups can run concurrently on the side streams
template <typename T>
int bprec(cheb_batch* B, const T* in, T* out, T* pa, T* pb) {
  int nact = 0;
  for (auto& g : B->pgroups) nact += g.hact.empty() ? 0 : 1;
  const bool fork = B->side_ok && nact > 1;
  int rc = fork ? side_fork(B) : CHEB_OK;
  if (rc) return rc;
  int i = 0;
  for (auto& g : B->pgroups) {
    if (g.hact.empty()) continue;
    hipStream_t st = fork ? B->side[i % kSide] : B->stream;
    ++i;
    rc = precond_apply_batch<T>(B->plans[g.rep], in, out, g.doffs, g.dsys, B->dkc, (int)g.hact.size(), B->P,
                                pa + g.pack_off, pb + g.pack_off, st);
    if (rc) break;
  }
  if (fork) {
    const int rj = side_join(B, i);
    if (!rc) rc = rj;
  }
  return rc;
}

// Autotuner of the batched operator: for every matrix-core size group not yet
// tuned in this precision, time the group's three-pass apply over all its
// members with each tile shape (HIP events, 4 applies after a warm-up) and
// keep the faster shape for the group's launches.
template <typename T>
int btune(cheb_batch* B, const T* K, const T* x, T* y) {
  const int pi = sizeof(T) == sizeof(double) ? 0 : 1;
  bool need = false;
  for (auto& g : B->groups) need = need || (g.dense && g.shape[pi] < 0);
  if (!need) return CHEB_OK;
  int rc = set_active(B, std::vector<char>(B->nprob, 1));
  if (rc) return rc;
  hipEvent_t e0, e1;
  rc = hip_check(hipEventCreate(&e0), "hipEventCreate");
  if (rc) return rc;
  rc = hip_check(hipEventCreate(&e1), "hipEventCreate");
  if (rc) {
    (void)hipEventDestroy(e0);
    return rc;
  }
  for (auto& g : B->groups) {
    if (!g.dense || g.shape[pi] >= 0 || rc) continue;
    cheb_plan* rep = B->plans[g.rep];
    const int nm = (int)g.hact.size();
    auto run = [&]() -> int {
      for (int pass = 0; pass < 3; ++pass) {
        const int r = launch_dense_batch<T>(rep, 2 - pass, pass == 0, K, x, y, g.dsys, g.dact, nm, B->stream);
        if (r) return r;
      }
      return CHEB_OK;
    };
    float best = 1e30f;
    int bv = 0;
    for (int v = 0; v < 2 && !rc; ++v) {
      for (int a = 0; a < 3; ++a) rep->dense_var[a][pi] = v;
      rc = run();
      if (!rc) rc = hip_check(hipEventRecord(e0, B->stream), "hipEventRecord");
      for (int r = 0; r < 4 && !rc; ++r) rc = run();
      if (!rc) rc = hip_check(hipEventRecord(e1, B->stream), "hipEventRecord");
      if (!rc) rc = hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
      float ms = 0.f;
      if (!rc) rc = hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
      if (rc) break;
      g.tuned_us[pi][v] = 1e3f * ms / 4.f;
      if (ms < best) {
        best = ms;
        bv = v;
      }
    }
    if (rc) break;
    for (int a = 0; a < 3; ++a) rep->dense_var[a][pi] = bv;
    g.shape[pi] = bv;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

enum { RUN = -100 };

// Lockstep LGMRES on A x = b for the systems with state[s] == RUN.  On return
// every such system has a final state (CHEB_OK, CHEB_NOT_CONVERGED or
// CHEB_STAGNATED), resid[s] its last true residual norm and mv[s] its matvecs.
template <typename T>
int blgmres(cheb_batch* B, const T* K, const T* b, T* x, bool x_zero, const std::vector<double>& tol, int maxmv,
            BKrylov<T>& kw, BScratch& sc, std::vector<int>& state, std::vector<double>& resid, std::vector<int>& mv,
            std::vector<int>& restarts, double stall, bool prec) {
  const int ns = B->nprob, m = kw.m, kmax = kw.k, cols = m + kmax;
  std::vector<std::vector<double>> H(ns), cs(ns), sn(ns), g(ns), yv(ns);
  std::vector<double> beta(ns, 0.0), beta_prev(ns, HUGE_VAL), hn(ns, 0.0);
  std::vector<int> jend(ns, 0);
  std::vector<int> zslot;
  std::vector<double> dots, coef((size_t)ns * kMaxCoef), scal((size_t)ns * 8);
  bool first = true;
  int rc;
  auto Hm = [&](int s, int i, int j) -> double& { return H[s][(size_t)i * cols + j]; };
  for (;;) {
    std::vector<char> on(ns, 0);
    int nrun = 0;
    for (int s = 0; s < ns; ++s)
      if (state[s] == RUN) on[s] = 1, ++nrun;
    if (!nrun) return CHEB_OK;
    rc = set_active(B, on);
    if (rc) return rc;
    // true residual into V_0
    T* v0 = kw.V;
    if (first && x_zero) {
      std::fill(scal.begin(), scal.end(), 0.0);
      for (int s = 0; s < ns; ++s) scal[(size_t)s * 8] = 1.0;
      rc = upload(B, B->dscal, scal.data(), scal.size(), 0);
      if (!rc) rc = baxpby<T, T>(B, v0, b, 0, -1);
    } else {
      rc = bapply<T>(B, K, x, v0);
      std::fill(scal.begin(), scal.end(), 0.0);
      for (int s = 0; s < ns; ++s) {
        scal[(size_t)s * 8] = 1.0;
        scal[(size_t)s * 8 + 1] = -1.0;
        if (on[s]) mv[s]++;
      }
      if (!rc) rc = upload(B, B->dscal, scal.data(), scal.size(), 0);
      if (!rc) rc = baxpby<T, T>(B, v0, b, 0, 1);
    }
    if (rc) return rc;
    first = false;
    rc = bdots<T>(B, nullptr, 0, 0, v0, sc, dots);
    if (rc) return rc;
    int ncyc = 0;
    for (int s = 0; s < ns; ++s) {
      if (!on[s]) continue;
      const double bb = dots[(size_t)s * kMaxCoef];
      beta[s] = std::sqrt(bb > 0 ? bb : 0.0);
      resid[s] = beta[s];
      if (!std::isfinite(beta[s])) state[s] = CHEB_NOT_CONVERGED;
      else if (!(beta[s] > tol[s])) state[s] = CHEB_OK;
      else if (mv[s] >= maxmv) state[s] = CHEB_NOT_CONVERGED;
      else if (stall > 0.0 && beta[s] > stall * beta_prev[s]) state[s] = CHEB_STAGNATED;
      beta_prev[s] = beta[s];
      if (state[s] == RUN) ++ncyc;
      else on[s] = 0;
    }
    if (!ncyc) return CHEB_OK;
    rc = set_active(B, on);
    if (rc) return rc;
    std::fill(scal.begin(), scal.end(), 0.0);
    for (int s = 0; s < ns; ++s) {
      scal[(size_t)s * 8] = on[s] ? 1.0 / beta[s] : 0.0;
      if (on[s]) {
        H[s].assign((size_t)(cols + 1) * cols, 0.0);
        cs[s].assign(cols, 0.0);
        sn[s].assign(cols, 0.0);
        g[s].assign(cols + 1, 0.0);
        g[s][0] = beta[s];
        jend[s] = 0;
      }
    }
    rc = upload(B, B->dscal, scal.data(), scal.size(), 0);
    if (!rc) rc = baxpby<T, T>(B, v0, v0, 0, -1);
    if (rc) return rc;
    std::vector<char> cyc = on;  // systems still extending the Krylov space this cycle
    const int jmax = m + (int)zslot.size();
    for (int j = 0; j < jmax; ++j) {
      const T* u = j < m ? kw.V + (size_t)j * kw.ld : kw.Z + (size_t)zslot[j - m] * kw.ld;
      if (prec) {
        rc = bprec<T>(B, u, kw.wp, kw.pa, kw.pb);
        if (rc) return rc;
        u = kw.wp;
      }
      rc = bapply<T>(B, K, u, kw.w);
      if (rc) return rc;
      for (int s = 0; s < ns; ++s)
        if (cyc[s]) mv[s]++;
      rc = bdots<T>(B, kw.V, kw.ld, j + 1, kw.w, sc, dots);
      if (rc) return rc;
      bool reorth = false;
      std::vector<double> hh2(ns, 0.0);
      for (int s = 0; s < ns; ++s) {
        if (!cyc[s]) continue;
        const double* d = &dots[(size_t)s * kMaxCoef];
        double h2 = d[j + 1];
        for (int i = 0; i <= j; ++i) {
          Hm(s, i, j) = d[i];
          h2 -= d[i] * d[i];
        }
        hh2[s] = h2;
        if (!(h2 > kReorthEta2 * d[j + 1])) reorth = true;
      }
      T* vnext = kw.V + (size_t)(j + 1) * kw.ld;
      std::fill(coef.begin(), coef.end(), 0.0);
      std::fill(scal.begin(), scal.end(), 0.0);
      for (int s = 0; s < ns; ++s)
        if (cyc[s])
          for (int i = 0; i <= j; ++i) coef[(size_t)s * kMaxCoef + i] = dots[(size_t)s * kMaxCoef + i];
      if (reorth) {
        // cancellation somewhere: a second classical Gram-Schmidt pass for all
        for (int s = 0; s < ns; ++s) scal[(size_t)s * 8] = cyc[s] ? 1.0 : 0.0;
        rc = upload(B, B->dcoef, coef.data(), coef.size(), 0);
        if (!rc) rc = upload(B, B->dscal, scal.data(), scal.size(), 1);
        if (!rc) rc = bupdate<T>(B, kw.V, kw.ld, j + 1, kw.w, kw.w);
        if (!rc) rc = bdots<T>(B, kw.V, kw.ld, j + 1, kw.w, sc, dots);
        if (rc) return rc;
        for (int s = 0; s < ns; ++s) {
          if (!cyc[s]) continue;
          const double* d = &dots[(size_t)s * kMaxCoef];
          double h2 = d[j + 1];
          for (int i = 0; i <= j; ++i) {
            Hm(s, i, j) += d[i];
            h2 -= d[i] * d[i];
            coef[(size_t)s * kMaxCoef + i] = d[i];
          }
          hh2[s] = h2;
        }
      }
      for (int s = 0; s < ns; ++s) {
        hn[s] = cyc[s] && hh2[s] > 0 ? std::sqrt(hh2[s]) : 0.0;
        scal[(size_t)s * 8] = hn[s] > 0 ? 1.0 / hn[s] : 0.0;
      }
      rc = upload(B, B->dcoef, coef.data(), coef.size(), 0);
      if (!rc) rc = upload(B, B->dscal, scal.data(), scal.size(), 1);
      if (!rc) rc = bupdate<T>(B, kw.V, kw.ld, j + 1, kw.w, vnext);
      if (rc) return rc;
      bool any = false;
      for (int s = 0; s < ns; ++s) {
        if (!cyc[s]) continue;
        Hm(s, j + 1, j) = hn[s];
        for (int i = 0; i < j; ++i) {
          const double a = Hm(s, i, j), bb = Hm(s, i + 1, j);
          Hm(s, i, j) = cs[s][i] * a + sn[s][i] * bb;
          Hm(s, i + 1, j) = -sn[s][i] * a + cs[s][i] * bb;
        }
        const double a = Hm(s, j, j), bb = Hm(s, j + 1, j);
        const double r = std::hypot(a, bb);
        cs[s][j] = r == 0.0 ? 1.0 : a / r;
        sn[s][j] = r == 0.0 ? 0.0 : bb / r;
        Hm(s, j, j) = r;
        Hm(s, j + 1, j) = 0.0;
        g[s][j + 1] = -sn[s][j] * g[s][j];
        g[s][j] = cs[s][j] * g[s][j];
        jend[s] = j + 1;
        const double est = std::fabs(g[s][j + 1]);
        const bool breakdown = !(bb > 1e-300) || !(r > 0);
        if (est <= tol[s] || mv[s] >= maxmv || breakdown) cyc[s] = 0;
        else any = true;
      }
      if (!any) break;
      rc = set_active(B, cyc);
      if (rc) return rc;
    }
    // per-system least squares y = R^{-1} g and the correction
    int nvmax = 0, jmaxend = 0;
    std::fill(coef.begin(), coef.end(), 0.0);
    for (int s = 0; s < ns; ++s) {
      if (!on[s]) continue;
      yv[s].assign(cols, 0.0);
      for (int i = jend[s] - 1; i >= 0; --i) {
        double t = g[s][i];
        for (int l = i + 1; l < jend[s]; ++l) t -= Hm(s, i, l) * yv[s][l];
        yv[s][i] = Hm(s, i, i) != 0.0 ? t / Hm(s, i, i) : 0.0;
      }
      for (int i = 0; i < jend[s]; ++i) coef[(size_t)s * kMaxCoef + i] = yv[s][i];
      nvmax = std::max(nvmax, std::min(jend[s], m));
      jmaxend = std::max(jmaxend, jend[s]);
    }
    // every system of the cycle forms its correction, including those that
    // stopped extending the space early
    rc = set_active(B, on);
    if (!rc) rc = upload(B, B->dcoef, coef.data(), coef.size(), 0);
    if (!rc) rc = blincomb<T>(B, kw.V, kw.ld, nvmax, 0, kw.w, 0);
    for (int i = m; i < jmaxend && !rc; ++i)
      rc = blincomb<T>(B, kw.Z + (size_t)zslot[i - m] * kw.ld, kw.ld, 1, i, kw.w, 1);
    if (rc) return rc;
    std::fill(scal.begin(), scal.end(), 0.0);
    for (int s = 0; s < ns; ++s) {
      scal[(size_t)s * 8] = on[s] ? 1.0 : 0.0;
      scal[(size_t)s * 8 + 1] = 1.0;
    }
    rc = upload(B, B->dscal, scal.data(), scal.size(), 1);
    if (rc) return rc;
    if (prec) {
      rc = bprec<T>(B, kw.w, kw.wp, kw.pa, kw.pb);
      if (!rc) rc = baxpby<T, T>(B, x, kw.wp, 0, 1);
    } else {
      rc = baxpby<T, T>(B, x, kw.w, 0, 1);
    }
    if (rc) return rc;
    if (kmax > 0) {
      int slot;
      if ((int)zslot.size() < kmax) {
        slot = (int)zslot.size();
      } else {
        slot = zslot.back();
        zslot.pop_back();
      }
      rc = hip_check(hipMemcpyAsync(kw.Z + (size_t)slot * kw.ld, kw.w, B->P * sizeof(T), hipMemcpyDeviceToDevice,
                                    B->stream),
                     "hipMemcpyAsync(D2D)");
      if (rc) return rc;
      zslot.insert(zslot.begin(), slot);
    }
    rc = bsync(B);
    if (rc) return rc;
    for (int s = 0; s < ns; ++s)
      if (on[s]) restarts[s]++;
  }
}

}  // namespace
}  // namespace cheb

using namespace cheb;

extern "C" {

int cheb_batch_create(const cheb_grid* grids, int32_t nprob, int32_t precision, void* stream, cheb_batch** out) {
  if (!grids || nprob <= 0 || !out) {
    set_error("invalid argument");
    return CHEB_ERR_INVALID_ARG;
  }
  if (precision != CHEB_F64 && precision != CHEB_MIXED) {
    set_error("batched solves run in CHEB_F64 or CHEB_MIXED");
    return CHEB_ERR_INVALID_ARG;
  }
  // systems of a group share one plan's boundary constants, which carry no
  // per-system Robin coefficient
  for (int s = 0; s < nprob; ++s)
    for (int f = 0; f < 6; ++f)
      if (grids[s].robin[f] != 0.0) {
        set_error("batched solves take Robin coefficient 0 on every face");
        return CHEB_ERR_UNSUPPORTED;
      }
  cheb_batch* B = new (std::nothrow) cheb_batch();
  if (!B) {
    set_error("out of host memory");
    return CHEB_ERR_INVALID_ARG;
  }
  B->nprob = nprob;
  B->prec = precision;
  B->stream = (hipStream_t)stream;
  B->ws = nullptr;
  B->ws_bytes = 0;
  B->side_ok = 0;
  int rc = CHEB_OK;
  auto fail = [&](int code) {
    cheb_batch_destroy(B);
    return code;
  };
  size_t P = 0;
  for (int s = 0; s < nprob; ++s) {
    cheb_plan* p = nullptr;
    rc = cheb_plan_create(&grids[s], precision, stream, &p);
    if (rc) return fail(rc);
    B->plans.push_back(p);
    B->off.push_back(P);
    B->npts.push_back(p->npts);
    P += round_up(p->npts, 64);
  }
  B->P = P;
  // apply groups: identical sizes and boxes (the face types may differ)
  auto same_box = [&](int a, int b) {
    for (int d = 0; d < 3; ++d)
      if (grids[a].n[d] != grids[b].n[d] || grids[a].lo[d] != grids[b].lo[d] || grids[a].hi[d] != grids[b].hi[d])
        return false;
    return true;
  };
  for (int s = 0; s < nprob; ++s) {
    bool placed = false;
    for (auto& g : B->groups)
      if (same_box(g.rep, s)) {
        g.members.push_back(s);
        placed = true;
        break;
      }
    if (!placed) {
      ApplyGroup g;
      g.rep = s;
      g.members.push_back(s);
      const cheb_plan* p = B->plans[s];
      g.dense = p->dd_ok[0] && p->dd_ok[1] && p->dd_ok[2] && p->ax[0].N == p->ax[1].N && p->ax[1].N == p->ax[2].N;
      B->groups.push_back(g);
    }
    bool pplaced = false;
    for (auto& g : B->pgroups)
      if (same_box(g.rep, s) && std::memcmp(grids[g.rep].bc, grids[s].bc, sizeof(grids[s].bc)) == 0) {
        g.members.push_back(s);
        pplaced = true;
        break;
      }
    if (!pplaced) {
      PrecGroup g;
      g.rep = s;
      g.members.push_back(s);
      B->pgroups.push_back(g);
    }
  }
  for (auto& g : B->groups) {
    const size_t nm = g.members.size();
    std::vector<DenseSys> tab(nm);
    for (size_t k = 0; k < nm; ++k) {
      tab[k].off = (long long)B->off[g.members[k]];
      tab[k].koff = tab[k].off;
      tab[k].bcmask = bc_mask(grids[g.members[k]].bc);
      tab[k].pad_ = 0;
    }
    g.htab = tab;
    if (!rc) rc = hip_check(hipMalloc((void**)&g.dsys, nm * sizeof(DenseSys)), "hipMalloc(batch table)");
    if (!rc) rc = hip_check(hipMalloc((void**)&g.dact, nm * sizeof(int)), "hipMalloc(batch table)");
    if (!rc) rc = hip_check(hipMemcpy(g.dsys, tab.data(), nm * sizeof(DenseSys), hipMemcpyHostToDevice), "hipMemcpy");
  }
  size_t pack = 0;
  for (auto& g : B->pgroups) {
    const size_t nm = g.members.size();
    if (!rc) rc = hip_check(hipMalloc((void**)&g.doffs, nm * sizeof(long long)), "hipMalloc(batch table)");
    if (!rc) rc = hip_check(hipMalloc((void**)&g.dsys, nm * sizeof(int)), "hipMalloc(batch table)");
    // room for every member's packed interior; the regions add up to at most P
    const cheb_grid& gr = grids[g.rep];
    g.pack_off = pack;
    pack += round_up((size_t)(gr.n[0] - 2) * (gr.n[1] - 2) * (gr.n[2] - 2) * nm, 64);
  }
  // side streams and their fork / join events (without them the groups run in
  // order on the batch's stream)
  {
    int made = 0;
    bool ok = hipEventCreateWithFlags(&B->ev_fork, hipEventDisableTiming) == hipSuccess;
    for (; ok && made < kSide; ++made) {
      if (hipStreamCreateWithFlags(&B->side[made], hipStreamNonBlocking) != hipSuccess) break;
      if (hipEventCreateWithFlags(&B->ev_join[made], hipEventDisableTiming) != hipSuccess) {
        (void)hipStreamDestroy(B->side[made]);
        break;
      }
    }
    if (ok && made == kSide) {
      B->side_ok = 1;
    } else {
      for (int k = 0; k < made; ++k) {
        (void)hipStreamDestroy(B->side[k]);
        (void)hipEventDestroy(B->ev_join[k]);
      }
      if (ok) (void)hipEventDestroy(B->ev_fork);
      (void)hipGetLastError();
    }
  }
  // chunk table of the segmented kernels
  std::vector<int> chs, chl, c0(nprob), nc(nprob);
  std::vector<long long> chb;
  for (int s = 0; s < nprob; ++s) {
    c0[s] = (int)chs.size();
    for (size_t b = 0; b < B->npts[s]; b += kChunk) {
      chs.push_back(s);
      chb.push_back((long long)(B->off[s] + b));
      chl.push_back((int)std::min<size_t>(kChunk, B->npts[s] - b));
    }
    nc[s] = (int)chs.size() - c0[s];
  }
  B->nchunks = (int)chs.size();
  B->ch_sys = nullptr;
  B->ch_beg = nullptr;
  B->ch_len = nullptr;
  B->sys_c0 = B->sys_nc = nullptr;
  B->chl = nullptr;
  B->nchl = 0;
  B->sys_c0_h = c0;
  B->sys_nc_h = nc;
  B->dcoef = B->dscal = B->dkc = nullptr;
  B->dflag = nullptr;
  B->hpin = nullptr;
  if (!rc) rc = hip_check(hipMalloc((void**)&B->ch_sys, chs.size() * sizeof(int)), "hipMalloc(chunks)");
  if (!rc) rc = hip_check(hipMalloc((void**)&B->ch_beg, chb.size() * sizeof(long long)), "hipMalloc(chunks)");
  if (!rc) rc = hip_check(hipMalloc((void**)&B->ch_len, chl.size() * sizeof(int)), "hipMalloc(chunks)");
  if (!rc) rc = hip_check(hipMalloc((void**)&B->chl, chs.size() * sizeof(int)), "hipMalloc(chunks)");
  if (!rc) rc = hip_check(hipMalloc((void**)&B->sys_c0, nprob * sizeof(int)), "hipMalloc(chunks)");
  if (!rc) rc = hip_check(hipMalloc((void**)&B->sys_nc, nprob * sizeof(int)), "hipMalloc(chunks)");
  if (!rc) rc = hip_check(hipMalloc((void**)&B->dcoef, (size_t)nprob * kMaxCoef * sizeof(double)), "hipMalloc");
  if (!rc) rc = hip_check(hipMalloc((void**)&B->dscal, (size_t)nprob * 8 * sizeof(double)), "hipMalloc");
  if (!rc) rc = hip_check(hipMalloc((void**)&B->dkc, (size_t)nprob * sizeof(double)), "hipMalloc");
  if (!rc) rc = hip_check(hipMalloc((void**)&B->dflag, sizeof(int)), "hipMalloc");
  if (!rc)
    rc = hip_check(hipHostMalloc((void**)&B->hpin, (size_t)3 * nprob * (kMaxCoef + 8) * sizeof(double),
                                 hipHostMallocDefault),
                   "hipHostMalloc");
  if (!rc) rc = hip_check(hipMemcpy(B->ch_sys, chs.data(), chs.size() * sizeof(int), hipMemcpyHostToDevice), "hipMemcpy");
  if (!rc) rc = hip_check(hipMemcpy(B->ch_beg, chb.data(), chb.size() * sizeof(long long), hipMemcpyHostToDevice), "hipMemcpy");
  if (!rc) rc = hip_check(hipMemcpy(B->ch_len, chl.data(), chl.size() * sizeof(int), hipMemcpyHostToDevice), "hipMemcpy");
  if (!rc) rc = hip_check(hipMemcpy(B->sys_c0, c0.data(), nprob * sizeof(int), hipMemcpyHostToDevice), "hipMemcpy");
  if (!rc) rc = hip_check(hipMemcpy(B->sys_nc, nc.data(), nprob * sizeof(int), hipMemcpyHostToDevice), "hipMemcpy");
  if (rc) return fail(rc);
  *out = B;
  return CHEB_OK;
}

int cheb_batch_workspace_bytes(const cheb_batch* batch, const cheb_solve_opts* opts, size_t* bytes) {
  if (!batch || !bytes) {
    set_error("null argument");
    return CHEB_ERR_INVALID_ARG;
  }
  BWS w;
  *bytes = carve_batch(const_cast<cheb_batch*>(batch), bparams(opts), nullptr, w);
  return CHEB_OK;
}

int cheb_batch_set_workspace(cheb_batch* batch, void* dev_ptr, size_t bytes) {
  if (!batch) {
    set_error("null batch");
    return CHEB_ERR_INVALID_ARG;
  }
  if (dev_ptr && ((uintptr_t)dev_ptr % 256) != 0) {
    set_error("workspace must be 256-byte aligned");
    return CHEB_ERR_WORKSPACE;
  }
  batch->ws = dev_ptr;
  batch->ws_bytes = dev_ptr ? bytes : 0;
  return CHEB_OK;
}

int cheb_batch_set_stream(cheb_batch* batch, void* stream) {
  if (!batch) {
    set_error("null batch");
    return CHEB_ERR_INVALID_ARG;
  }
  batch->stream = (hipStream_t)stream;
  for (cheb_plan* p : batch->plans) cheb_plan_set_stream(p, stream);
  return CHEB_OK;
}

int cheb_batch_solve(cheb_batch* batch, const void* const* K, const void* const* f, const void* const* g_faces,
                     void* const* u_inout, const cheb_solve_opts* opts, cheb_solve_info* infos) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!batch || !K || !f || !g_faces || !u_inout) {
    set_error("null argument");
    return CHEB_ERR_INVALID_ARG;
  }
  cheb_batch* B = batch;
  const int ns = B->nprob;
  for (int s = 0; s < ns; ++s)
    if (!K[s] || !f[s] || !g_faces[s] || !u_inout[s]) {
      set_error("null field pointer");
      return CHEB_ERR_INVALID_ARG;
    }
  const BParams bp = bparams(opts);
  if (bp.m < 1 || bp.m + bp.k + 2 > 72 || bp.k < 0 || bp.k > 6) {
    set_error("inner_m must be in [1, 64] and outer_k in [0, 6]");
    return CHEB_ERR_INVALID_ARG;
  }
  BWS w;
  const size_t need = carve_batch(B, bp, nullptr, w);
  if (!B->ws || B->ws_bytes < need) {
    set_error("workspace missing or too small (see cheb_batch_workspace_bytes)");
    return CHEB_ERR_WORKSPACE;
  }
  carve_batch(B, bp, (char*)B->ws, w);
  hipStream_t st = B->stream;
  int rc = CHEB_OK;
  for (cheb_plan* p : B->plans) cheb_plan_set_stream(p, B->stream);
  // validate K, pack it, and form the reduced right-hand sides
  rc = hip_check(hipMemsetAsync(B->dflag, 0, sizeof(int), st), "hipMemsetAsync");
  for (int s = 0; s < ns && !rc; ++s) rc = check_positive_finite((const double*)K[s], B->npts[s], B->dflag, st);
  int* hf = (int*)B->hpin;
  if (!rc) rc = hip_check(hipMemcpyAsync(hf, B->dflag, sizeof(int), hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
  if (!rc) rc = bsync(B);
  if (rc) return rc;
  if (*hf) {
    set_error("conductivity must be finite and positive at every node");
    return CHEB_ERR_BAD_INPUT;
  }
  rc = fill<double>(w.K64, 1.0, round_up(B->P, 64), st);
  if (!rc) rc = fill<double>(w.bt, 0.0, round_up(B->P, 64), st);
  if (!rc) rc = fill<double>(w.x, 0.0, round_up(B->P, 64), st);
  // systems given the same K (and grid size) share one packed copy, so a
  // batched pass over them reads the same conductivity lines
  B->koff.assign(ns, 0);
  for (int s = 0; s < ns; ++s) {
    B->koff[s] = B->off[s];
    for (int q = 0; q < s; ++q)
      if (K[q] == K[s] && B->npts[q] == B->npts[s] && B->koff[q] == B->off[q]) {
        B->koff[s] = B->off[q];
        break;
      }
  }
  for (auto& g : B->groups) {
    bool changed = false;
    for (size_t k = 0; k < g.members.size(); ++k) {
      const long long ko = (long long)B->koff[g.members[k]];
      changed = changed || g.htab[k].koff != ko;
      g.htab[k].koff = ko;
    }
    if (changed && g.dsys)
      rc = hip_check(hipMemcpyAsync(g.dsys, g.htab.data(), g.htab.size() * sizeof(DenseSys), hipMemcpyHostToDevice, st),
                     "hipMemcpyAsync(batch table)");
    if (!rc) rc = bsync(B);  // the host table is pageable: the copy completes before it changes
    if (rc) return rc;
  }
  for (int s = 0; s < ns && !rc; ++s) {
    cheb_plan* p = B->plans[s];
    const size_t o = B->off[s];
    const double* Ks = (const double*)K[s];
    if (B->koff[s] == o) rc = copy_scale<double>(w.K64 + o, Ks, 1.0, p->npts, st);
    if (!rc) rc = fill<double>(w.t1 + o, 0.0, p->npts, st);
    if (!rc) rc = lift_full<double>(p, w.t1 + o, (const double*)g_faces[s], st);
    if (!rc) rc = apply_t<double>(p, Ks, w.t1 + o, w.bt + o, 0, st);
    if (!rc) rc = rhs_reduced<double>(w.bt + o, (const double*)f[s], p->g.n, st);
    if (!rc && bp.warm) {
      rc = copy_scale<double>(w.x + o, (const double*)u_inout[s], 1.0, p->npts, st);
      if (!rc) rc = mask_interior<double>(w.x + o, p->g.n, st);
    }
  }
  if (rc) return rc;
  if (bp.precond) {
    std::vector<double> kc(ns);
    // a group's batched contractions read only its representative's factors
    for (const auto& g : B->pgroups)
      if (!rc) rc = precond_setup(B->plans[g.rep]);
    for (int s = 0; s < ns && !rc; ++s)
      rc = vsum<double>((const double*)K[s], B->npts[s], w.sc.partials, w.sc.dots + s, st);
    double* hp = B->hpin;
    if (!rc) rc = hip_check(hipMemcpyAsync(hp, w.sc.dots, ns * sizeof(double), hipMemcpyDeviceToHost, st), "D2H");
    if (!rc) rc = bsync(B);
    if (rc) return rc;
    for (int s = 0; s < ns; ++s) kc[s] = hp[s] / double(B->npts[s]);
    rc = hip_check(hipMemcpyAsync(B->dkc, kc.data(), ns * sizeof(double), hipMemcpyHostToDevice, st), "H2D");
    if (!rc) rc = bsync(B);
    if (rc) return rc;
  }
  std::vector<int> state(ns, RUN), mv(ns, 0), mv32(ns, 0), restarts(ns, 0), irs(ns, 0);
  std::vector<double> resid(ns, 0.0), bnorm(ns, 0.0), tol(ns, 0.0);
  std::vector<double> dots;
  rc = set_active(B, std::vector<char>(ns, 1));
  if (!rc) rc = bdots<double>(B, nullptr, 0, 0, w.bt, w.sc, dots);
  if (rc) return rc;
  for (int s = 0; s < ns; ++s) {
    bnorm[s] = std::sqrt(std::max(0.0, dots[(size_t)s * kMaxCoef]));
    tol[s] = std::fmax(bp.rtol * bnorm[s], bp.atol);
    if (bnorm[s] == 0.0) state[s] = CHEB_OK;
  }
  // tile shapes of the size groups (timed on the first solve in each precision;
  // the outputs land in scratch fields that are rewritten before use)
  rc = btune<double>(B, w.K64, w.bt, w.t1);
  if (rc) return rc;
  if (B->prec == CHEB_F64) {
    rc = blgmres<double>(B, w.K64, w.bt, w.x, !bp.warm, tol, bp.maxiter, w.kw64, w.sc, state, resid, mv, restarts,
                         0.0, bp.precond);
  } else {
    // FP64 refinement around lockstep FP32 inner solves
    rc = cast_f64_f32(w.K32, w.K64, 1.0, round_up(B->P, 64), st);
    if (!rc) rc = cast_f64_f32(w.b32, w.bt, 1.0, round_up(B->P, 64), st);
    if (!rc) rc = btune<float>(B, w.K32, w.b32, w.d32);
    std::vector<double> prev(ns, HUGE_VAL), rho(ns, 0.0), scal((size_t)ns * 8, 0.0);
    std::vector<int> slow(ns, 0);
    std::vector<char> on(ns, 0);
    for (int it = 0; !rc; ++it) {
      for (int s = 0; s < ns; ++s) on[s] = state[s] == RUN;
      rc = set_active(B, on);
      if (!rc) rc = bapply<double>(B, w.K64, w.x, w.r);
      std::fill(scal.begin(), scal.end(), 0.0);
      for (int s = 0; s < ns; ++s) {
        scal[(size_t)s * 8] = 1.0;
        scal[(size_t)s * 8 + 1] = -1.0;
        if (on[s]) mv[s]++;
      }
      if (!rc) rc = upload(B, B->dscal, scal.data(), scal.size(), 0);
      if (!rc) rc = baxpby<double, double>(B, w.r, w.bt, 0, 1);
      if (!rc) rc = bdots<double>(B, nullptr, 0, 0, w.r, w.sc, dots);
      if (rc) break;
      int nrun = 0;
      for (int s = 0; s < ns; ++s) {
        if (!on[s]) continue;
        rho[s] = std::sqrt(std::max(0.0, dots[(size_t)s * kMaxCoef]));
        resid[s] = rho[s];
        if (!std::isfinite(rho[s])) {
          state[s] = CHEB_NOT_CONVERGED;
        } else if (!(rho[s] > tol[s])) {
          state[s] = CHEB_OK;
        } else if (irs[s] >= bp.ir_max || mv[s] >= bp.maxiter) {
          state[s] = CHEB_NOT_CONVERGED;
        } else {
          if (rho[s] > 0.5 * prev[s]) {
            if (++slow[s] >= 3) state[s] = CHEB_STAGNATED;
          } else {
            slow[s] = 0;
          }
          prev[s] = rho[s];
        }
        if (state[s] == RUN) ++nrun;
      }
      if (!nrun) break;
      // b32 = r / rho (zero for finished systems), d32 = 0
      std::fill(scal.begin(), scal.end(), 0.0);
      for (int s = 0; s < ns; ++s) scal[(size_t)s * 8] = state[s] == RUN ? 1.0 / rho[s] : 0.0;
      rc = upload(B, B->dscal, scal.data(), scal.size(), 1);
      if (!rc) rc = baxpby<float, double>(B, w.b32, w.r, 0, -1);
      if (!rc) rc = fill<float>(w.d32, 0.0, round_up(B->P, 64), st);
      if (rc) break;
      std::vector<int> istate(ns, CHEB_OK), imv(ns, 0);
      std::vector<double> ires(ns, 0.0), itol(ns, bp.ir_rtol);
      int budget = 1 << 30;
      for (int s = 0; s < ns; ++s)
        if (state[s] == RUN) {
          istate[s] = RUN;
          irs[s]++;
          budget = std::min(budget, bp.maxiter - mv[s]);
          // as the single-system refinement: the reduction still needed, not
          // below ir_inner_rtol
          itol[s] = std::fmax(bp.ir_rtol, 0.3 * tol[s] / rho[s]);
        }
      const int cap = 40 * (bp.m + bp.k + 1);
      budget = std::max(1, std::min(budget, cap));
      rc = blgmres<float>(B, w.K32, w.b32, w.d32, true, itol, budget, w.kw32, w.sc, istate, ires, imv, restarts,
                          0.9, bp.precond);
      if (rc) break;
      std::fill(scal.begin(), scal.end(), 0.0);
      for (int s = 0; s < ns; ++s) {
        mv[s] += imv[s];
        mv32[s] += imv[s];
        scal[(size_t)s * 8] = state[s] == RUN ? rho[s] : 0.0;
        scal[(size_t)s * 8 + 1] = 1.0;
      }
      // the inner solve leaves its own last active set behind: restore this step's
      for (int s2 = 0; s2 < ns; ++s2) on[s2] = state[s2] == RUN;
      rc = set_active(B, on);
      if (!rc) rc = upload(B, B->dscal, scal.data(), scal.size(), 0);
      if (!rc) rc = baxpby<double, float>(B, w.x, w.d32, 0, 1);
      if (!rc) rc = bsync(B);
    }
  }
  if (rc) return rc;
  // full-grid solutions
  for (int s = 0; s < ns && !rc; ++s) {
    cheb_plan* p = B->plans[s];
    rc = copy_scale<double>((double*)u_inout[s], w.x + B->off[s], 1.0, p->npts, st);
    if (!rc) rc = lift_full<double>(p, (double*)u_inout[s], (const double*)g_faces[s], st);
  }
  if (!rc) rc = bsync(B);
  if (rc) return rc;
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int worst = CHEB_OK;
  for (int s = 0; s < ns; ++s) {
    const int stt = state[s] == RUN ? CHEB_NOT_CONVERGED : state[s];
    if (infos) {
      cheb_solve_info inf{};
      inf.status = stt;
      inf.matvecs = mv[s];
      inf.matvecs_f32 = mv32[s];
      inf.restarts = restarts[s];
      inf.ir_steps = irs[s];
      inf.relres_final = bnorm[s] > 0 ? resid[s] / bnorm[s] : 0.0;
      inf.seconds = secs;
      infos[s] = inf;
    }
    worst = std::max(worst, stt);
  }
  return worst;
}

int cheb_batch_tile_shapes(const cheb_batch* batch, int32_t field_precision, int32_t* out, int32_t len) {
  if (!batch || (len > 0 && !out) || (field_precision != CHEB_F64 && field_precision != CHEB_F32)) {
    set_error("invalid argument");
    return CHEB_ERR_INVALID_ARG;
  }
  const int pi = field_precision == CHEB_F64 ? 0 : 1;
  int k = 0;
  for (const auto& g : batch->groups) {
    if (!g.dense) continue;
    const int vals[4] = {batch->plans[g.rep]->g.n[0], g.shape[pi], (int)(g.tuned_us[pi][0] * 1000.f),
                         (int)(g.tuned_us[pi][1] * 1000.f)};
    for (int q = 0; q < 4; ++q)
      if (k < len) out[k++] = vals[q];
  }
  return k / 4;
}

int cheb_batch_destroy(cheb_batch* batch) {
  if (!batch) return CHEB_OK;
  for (auto& g : batch->groups) {
    if (g.dsys) (void)hipFree(g.dsys);
    if (g.dact) (void)hipFree(g.dact);
  }
  for (auto& g : batch->pgroups) {
    if (g.doffs) (void)hipFree(g.doffs);
    if (g.dsys) (void)hipFree(g.dsys);
  }
  if (batch->ch_sys) (void)hipFree(batch->ch_sys);
  if (batch->ch_beg) (void)hipFree(batch->ch_beg);
  if (batch->ch_len) (void)hipFree(batch->ch_len);
  if (batch->chl) (void)hipFree(batch->chl);
  if (batch->sys_c0) (void)hipFree(batch->sys_c0);
  if (batch->sys_nc) (void)hipFree(batch->sys_nc);
  if (batch->dcoef) (void)hipFree(batch->dcoef);
  if (batch->dscal) (void)hipFree(batch->dscal);
  if (batch->dkc) (void)hipFree(batch->dkc);
  if (batch->dflag) (void)hipFree(batch->dflag);
  if (batch->hpin) (void)hipHostFree(batch->hpin);
  if (batch->side_ok) {
    for (int k = 0; k < kSide; ++k) {
      (void)hipStreamDestroy(batch->side[k]);
      (void)hipEventDestroy(batch->ev_join[k]);
    }
    (void)hipEventDestroy(batch->ev_fork);
  }
  for (cheb_plan* p : batch->plans) cheb_plan_destroy(p);
  delete batch;
  return CHEB_OK;
}

}  // extern "C"
