// Axis-pass kernel: for every pencil along one axis, y (+)= D_a (K * D_a u)
// with the boundary rows / boundary elimination of the chosen mode.
//
// Per pencil the derivative is the paper's transform route (Section 2.2,
// Algorithm 1), realised with a recurrence instead of the sine transform:
//   X = C u                  unnormalised DCT-I (FFT of the even extension)
//   w_j = c j eps_j X_j      c = -1/(N L_a) folds 1/N, the affine map and the
//                            ascending node order; eps = 1 at j = 0, N else 2
//   beta_k = sum_{j>k, j-k odd} w_j     derivative-coefficient recurrence
//   D u = C beta             back-transform (a DCT-I of the coefficients)
// applied twice with the pointwise flux K * D_a u in between (Algorithm 3).
// The transpose runs D^T = E C (c J) S^T E C E^{-1} (S^T: prefix sums).
//
// DCT-I of two real pencils at once: pencil A in the real part, pencil B in
// the imaginary part of one complex FFT of length L = 2N (four-step split
// L = R1*R2, register DFTs, one LDS exchange).  The even symmetry of the input
// makes columns n2 and R2-n2 of the exchange related, so only R2/2+1 columns
// are computed and stored.
#pragma once

#include "dev_common.h"
#include "pencil.h"

namespace cheb {

enum PassMode { MODE_FULL = 0, MODE_REDUCED = 1, MODE_TRANSPOSE = 2, MODE_DERIV = 3, MODE_DERIV_T = 4 };

template <typename T>
struct PassArgs {
  const T* u;
  const T* K;
  T* y;
  const T* drow0;  // row 0 of the ascending, scaled differentiation matrix (n entries)
  const T* drowN;  // row N
  int n[3];
  int axis;
  int N;      // n[axis] - 1
  int first;  // this pass initialises every row it owns ('='); later passes accumulate
  int bc[6];
  T cscale;   // -1 / (N * L_axis)
  T m00, m0N, mN0, mNN;  // corner entries of that matrix
  int npencils;
};

// ---------------------------------------------------------------------------
// Tile shape per transform size
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int pass_pencils(int N) {
  return N == 0 ? 16 : N <= 32 ? 64 : N <= 64 ? 32 : 16;
}
__host__ __device__ constexpr int pass_threads(int N) { return N >= 256 ? 256 : 128; }

struct PassLayout {
  int e_off, tw_off, sv_off, tmp_off, ends_off, base_off, flags_off, bytes, svs;
};

// LDS layout (bytes) of one tile; NC = compile-time N (0 = generic direct DCT).
template <typename T>
__host__ __device__ constexpr PassLayout pass_layout(int NC, int Nrt) {
  const int N = NC > 0 ? NC : Nrt;
  const int P = pass_pencils(NC);
  const int n = N + 1;
  const int svs = n + 1;
  PassLayout l{0, 0, 0, 0, 0, 0, 0, 0, svs};
  int off = 0;
  if (NC > 0) {
    const Split sp = fft_split(2 * N);
    const int EH = sp.r2 / 2 + 2;
    l.e_off = off;
    off += (P / 2) * sp.r1 * EH * 2 * (int)sizeof(T);
    l.tw_off = off;
    off += 2 * N * 2 * (int)sizeof(T);
    l.sv_off = off;
    off += P * svs * (int)sizeof(T);
    l.tmp_off = off;
  } else {
    l.sv_off = off;
    off += P * svs * (int)sizeof(T);
    l.tmp_off = off;
    off += P * svs * (int)sizeof(T);
    l.tw_off = off;  // cos(pi j / N), j < 2N
    off += 2 * N * (int)sizeof(T);
  }
  off = (off + 15) & ~15;
  l.ends_off = off;
  off += 4 * P * (int)sizeof(T);
  off = (off + 15) & ~15;
  l.base_off = off;
  off += P * 8;
  l.flags_off = off;
  off += P * 4;
  l.bytes = (off + 15) & ~15;
  return l;
}

// ---------------------------------------------------------------------------
// DCT-I of all pencils of the tile, in place in sv (pencil stride SVS).
// ---------------------------------------------------------------------------
template <typename T, int NC, int P, int NT>
__device__ __forceinline__ void dct_tile_fast(T* sv, cplx<T>* E, const cplx<T>* tw, int tid) {
  constexpr int N = NC, L = 2 * N, SVS = N + 2;
  constexpr Split sp = fft_split(L);
  constexpr int R1 = sp.r1, R2 = sp.r2, H = R2 / 2 + 1, EH = H + 1, Q = P / 2;
  static_assert(R1 > 0 && R2 % 2 == 0, "transform size not supported");
  // stage 1: columns n2 = 0..R2/2, DFT over n1, twiddle W_L^{n2 k1}
  for (int w = tid; w < Q * H; w += NT) {
    const int q = w / H, n2 = w - q * H;
    const T* a = sv + (2 * q) * SVS;
    const T* b = a + SVS;
    T re[R1], im[R1];
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) {
      const int m = R2 * n1 + n2;
      const int s = m <= N ? m : L - m;
      re[n1] = a[s];
      im[n1] = b[s];
    }
    DFT<R1>::run(re, im);
    cplx<T>* e = E + (q * R1) * EH + n2;
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      const cplx<T> t = tw[n2 * k1];
      cplx<T> v;
      v.x = re[k1] * t.x - im[k1] * t.y;
      v.y = re[k1] * t.y + im[k1] * t.x;
      e[k1 * EH] = v;
    }
  }
  __syncthreads();
  // stage 2: rows k1, DFT over n2 (columns > R2/2 from the mirrored row)
  for (int w = tid; w < Q * R1; w += NT) {
    const int q = w / R1, k1 = w - q * R1;
    const int k1p = k1 == 0 ? 0 : R1 - k1;
    const cplx<T>* e = E + (q * R1) * EH;
    T re[R2], im[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
      if (n2 <= R2 / 2) {
        const cplx<T> v = e[k1 * EH + n2];
        re[n2] = v.x;
        im[n2] = v.y;
      } else {
        const cplx<T> v = e[k1p * EH + (R2 - n2)];
        const T c = T(ct_cos2pi(n2, R2)), s = T(-ct_sin2pi(n2, R2));
        const T vr = v.x * c - v.y * s, vi = v.x * s + v.y * c;
        re[n2] = k1 ? vr : v.x;
        im[n2] = k1 ? vi : v.y;
      }
    }
    DFT<R2>::run(re, im);
    T* a = sv + (2 * q) * SVS;
    T* b = a + SVS;
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) {
      const int k = k1 + R1 * k2;
      if (k <= N) {
        a[k] = re[k2];
        b[k] = im[k2];
      }
    }
  }
  __syncthreads();
}

// Generic size: direct DCT-I sum with a cosine table (O(N^2) per pencil).
template <typename T, int P, int NT>
__device__ __forceinline__ void dct_tile_direct(T* sv, T* tmp, const T* ctab, int N, int tid) {
  const int n = N + 1, SVS = N + 2, L = 2 * N;
  for (int e = tid; e < P * n; e += NT) {
    const int pl = e / n, k = e - pl * n;
    const T* s = sv + pl * SVS;
    T acc = s[0] + ((k & 1) ? -s[N] : s[N]);
    int idx = 0;
    for (int m = 1; m < N; ++m) {
      idx += k;
      if (idx >= L) idx -= L;
      acc += T(2) * s[m] * ctab[idx];
    }
    tmp[pl * SVS + k] = acc;
  }
  __syncthreads();
  for (int e = tid; e < P * n; e += NT) {
    const int pl = e / n, k = e - pl * n;
    sv[pl * SVS + k] = tmp[pl * SVS + k];
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Coefficient-space recurrences on one pencil, G lanes per pencil.
// ---------------------------------------------------------------------------
template <typename T, int G>
__device__ __forceinline__ void recur_forward(T* pen, int N, T c, int g) {
  const int n = N + 1;
  const int C = (((n + G - 1) / G) + 1) & ~1;
  const int j0 = g * C < n ? g * C : n;
  const int j1 = j0 + C < n ? j0 + C : n;
  T t0 = T(0), t1 = T(0);
  for (int j = j0; j < j1; ++j) {
    const T w = pen[j] * T(j) * ((j == 0 || j == N) ? T(1) : T(2));
    if (j & 1) t1 += w; else t0 += w;
  }
  T r0 = group_suffix_excl<G>(t0, g);
  T r1 = group_suffix_excl<G>(t1, g);
  for (int j = j1 - 1; j >= j0; --j) {
    const T w = pen[j] * T(j) * ((j == 0 || j == N) ? T(1) : T(2));
    const T beta = (j & 1) ? r0 : r1;  // sum of w_i, i > j, i of the other parity
    pen[j] = c * beta;
    if (j & 1) r1 += w; else r0 += w;
  }
}

template <typename T, int G>
__device__ __forceinline__ void recur_transpose(T* pen, int N, T c, int g) {
  const int n = N + 1;
  const int C = (((n + G - 1) / G) + 1) & ~1;
  const int j0 = g * C < n ? g * C : n;
  const int j1 = j0 + C < n ? j0 + C : n;
  T t0 = T(0), t1 = T(0);
  for (int j = j0; j < j1; ++j) {
    const T t = pen[j] * ((j == 0 || j == N) ? T(1) : T(2));
    if (j & 1) t1 += t; else t0 += t;
  }
  T r0 = group_prefix_excl<G>(t0, g);
  T r1 = group_prefix_excl<G>(t1, g);
  for (int j = j0; j < j1; ++j) {
    const T t = pen[j] * ((j == 0 || j == N) ? T(1) : T(2));
    const T rho = (j & 1) ? r0 : r1;  // sum of t_k, k < j, k of the other parity
    pen[j] = c * T(j) * rho;
    if (j & 1) r1 += t; else r0 += t;
  }
}

// ---------------------------------------------------------------------------
// The pass kernel
// ---------------------------------------------------------------------------
template <typename T, int NC, int MODE>
__global__ __launch_bounds__(pass_threads(NC)) void k_axis_pass(PassArgs<T> a) {
  constexpr int P = pass_pencils(NC);
  constexpr int NT = pass_threads(NC);
  constexpr int G = NT / P;
  static_assert(NT % P == 0 && 64 % G == 0, "bad tile shape");
  extern __shared__ __align__(16) unsigned char smem[];
  const int N = NC > 0 ? NC : a.N;
  const int n = N + 1;
  const PassLayout lay = pass_layout<T>(NC, N);
  const int SVS = lay.svs;
  T* sv = (T*)(smem + lay.sv_off);
  T* ends = (T*)(smem + lay.ends_off);
  long long* base = (long long*)(smem + lay.base_off);
  int* flags = (int*)(smem + lay.flags_off);
  cplx<T>* E = (cplx<T>*)(smem + lay.e_off);
  cplx<T>* tw = (cplx<T>*)(smem + lay.tw_off);
  T* tmp = (T*)(smem + lay.tmp_off);
  T* ctab = (T*)(smem + lay.tw_off);

  const int tid = threadIdx.x;
  const int tile = xcd_swizzle(blockIdx.x, gridDim.x);
  const int p0 = tile * P;
  const int axis = a.axis;
  const int n0 = a.n[0], n1 = a.n[1], n2 = a.n[2];
  const long long stride = axis == 2 ? 1LL : axis == 1 ? (long long)n2 : (long long)n1 * n2;
  const bool contig = axis == 2;

  // twiddles W_L^j (fast path) or cos(pi j/N) (direct path)
  if (NC > 0) {
    for (int j = tid; j < 2 * N; j += NT) {
      double s, c;
      sincospi(double(j) / double(N), &s, &c);
      cplx<T> t;
      t.x = T(c);
      t.y = T(-s);
      tw[j] = t;
    }
  } else {
    for (int j = tid; j < 2 * N; j += NT) ctab[j] = T(cospi(double(j) / double(N)));
  }
  // pencil classification
  if (tid < P) {
    long long b = 0;
    flags[tid] = pencil_flags(axis, p0 + tid, a.npencils, a.n, a.bc, &b);
    base[tid] = b;
  }
  __syncthreads();

  // load the tile
  for (int e = tid; e < P * n; e += NT) {
    int pl, m;
    if (contig) { pl = e / n; m = e - pl * n; }
    else { m = e / P; pl = e - m * P; }
    const int fl = flags[pl];
    T v = T(0);
    if (fl & PF_VALID) {
      const bool ld = (MODE == MODE_FULL || MODE == MODE_DERIV || MODE == MODE_DERIV_T) || (fl & PF_TIN);
      if (ld) v = a.u[base[pl] + m * stride];
      if (MODE == MODE_DERIV_T && m != 0 && m != N) v *= T(0.5);
      if (MODE == MODE_REDUCED || MODE == MODE_TRANSPOSE) {
        if (m == 0 || m == N) v = T(0);
        else if (MODE == MODE_TRANSPOSE) v *= T(0.5);
      }
      if (MODE == MODE_FULL) {
        if (m == 0) ends[4 * pl + 0] = v;
        if (m == N) ends[4 * pl + 1] = v;
      }
    }
    sv[pl * SVS + m] = v;
  }
  __syncthreads();

  const int pp = tid / G, g = tid - pp * G;
  T* pen = sv + pp * SVS;

  if (MODE == MODE_REDUCED) {
    // homogeneous lift of the pencil's end values (Neumann rows, Section 2.3.1)
    T s0 = T(0), sN = T(0);
    for (int m = 1 + g; m < N; m += G) {
      const T v = pen[m];
      s0 += a.drow0[m] * v;
      sN += a.drowN[m] * v;
    }
    s0 = group_sum<G>(s0);
    sN = group_sum<G>(sN);
    const int fl = flags[pp];
    if (g == 0 && (fl & PF_TIN)) {
      const bool nlo = a.bc[2 * axis] == 1, nhi = a.bc[2 * axis + 1] == 1;
      T u0 = T(0), uN = T(0);
      if (nlo && nhi) {
        const T det = a.m00 * a.mNN - a.m0N * a.mN0;
        u0 = (-s0 * a.mNN + sN * a.m0N) / det;
        uN = (-sN * a.m00 + s0 * a.mN0) / det;
      } else if (nlo) {
        u0 = -s0 / a.m00;
      } else if (nhi) {
        uN = -sN / a.mNN;
      }
      pen[0] = u0;
      pen[N] = uN;
    }
    __syncthreads();
  }

  // first derivative (or its transpose)
  if constexpr (NC > 0) dct_tile_fast<T, NC, P, NT>(sv, E, tw, tid);
  else dct_tile_direct<T, P, NT>(sv, tmp, ctab, N, tid);
  if (MODE == MODE_TRANSPOSE || MODE == MODE_DERIV_T) recur_transpose<T, G>(pen, N, a.cscale, g);
  else recur_forward<T, G>(pen, N, a.cscale, g);
  __syncthreads();
  if constexpr (NC > 0) dct_tile_fast<T, NC, P, NT>(sv, E, tw, tid);
  else dct_tile_direct<T, P, NT>(sv, tmp, ctab, N, tid);

  if (MODE != MODE_DERIV && MODE != MODE_DERIV_T) {
    // pointwise flux K * D_a u (boundary nodes included)
    for (int e = tid; e < P * n; e += NT) {
      int pl, m;
      if (contig) { pl = e / n; m = e - pl * n; }
      else { m = e / P; pl = e - m * P; }
      const int fl = flags[pl];
      T v = sv[pl * SVS + m];
      if (MODE == MODE_FULL) {
        if (m == 0) ends[4 * pl + 2] = v;
        if (m == N) ends[4 * pl + 3] = v;
      }
      T k = T(0);
      if (fl & PF_VALID) k = a.K[base[pl] + m * stride];
      sv[pl * SVS + m] = v * k;
    }
    __syncthreads();
    // divergence part
    if constexpr (NC > 0) dct_tile_fast<T, NC, P, NT>(sv, E, tw, tid);
    else dct_tile_direct<T, P, NT>(sv, tmp, ctab, N, tid);
    if (MODE == MODE_TRANSPOSE) recur_transpose<T, G>(pen, N, a.cscale, g);
    else recur_forward<T, G>(pen, N, a.cscale, g);
    __syncthreads();
    if constexpr (NC > 0) dct_tile_fast<T, NC, P, NT>(sv, E, tw, tid);
    else dct_tile_direct<T, P, NT>(sv, tmp, ctab, N, tid);
  }

  if (MODE == MODE_TRANSPOSE) {
    // transposed lift: mu = M^{-T} [z_0, z_N]; interior -= mu0 D_{0,:} + muN D_{N,:}
    if (g == 0) {
      const bool nlo = a.bc[2 * axis] == 1, nhi = a.bc[2 * axis + 1] == 1;
      const T z0 = pen[0], zN = pen[N];
      T mu0 = T(0), muN = T(0);
      if (nlo && nhi) {
        const T det = a.m00 * a.mNN - a.m0N * a.mN0;
        mu0 = (z0 * a.mNN - zN * a.mN0) / det;
        muN = (zN * a.m00 - z0 * a.m0N) / det;
      } else if (nlo) {
        mu0 = z0 / a.m00;
      } else if (nhi) {
        muN = zN / a.mNN;
      }
      ends[4 * pp + 0] = mu0;
      ends[4 * pp + 1] = muN;
    }
    __syncthreads();
  }

  // store
  for (int e = tid; e < P * n; e += NT) {
    int pl, m;
    if (contig) { pl = e / n; m = e - pl * n; }
    else { m = e / P; pl = e - m * P; }
    const int fl = flags[pl];
    if (!(fl & PF_VALID)) continue;
    const long long ad = base[pl] + m * stride;
    T v = sv[pl * SVS + m];
    const bool isend = (m == 0 || m == N);
    if (MODE == MODE_DERIV) {
      a.y[ad] = v;
    } else if (MODE == MODE_DERIV_T) {
      a.y[ad] = isend ? v : T(2) * v;
    } else if (MODE == MODE_FULL) {
      if (!isend) {
        if (fl & PF_TIN) a.y[ad] = a.first ? v : a.y[ad] + v;
      } else {
        const bool own = (m == 0) ? (fl & PF_OWN_LO) : (fl & PF_OWN_HI);
        if (own) {
          const int bct = a.bc[2 * axis + (m == 0 ? 0 : 1)];
          T r;
          if (bct == 0) r = ends[4 * pl + (m == 0 ? 0 : 1)];
          else r = (m == 0) ? -ends[4 * pl + 2] : ends[4 * pl + 3];
          a.y[ad] = r;
        }
      }
    } else {
      if (!(fl & PF_TIN) || isend) {
        if (a.first) a.y[ad] = T(0);
      } else {
        if (MODE == MODE_TRANSPOSE)
          v = T(2) * v - ends[4 * pl + 0] * a.drow0[m] - ends[4 * pl + 1] * a.drowN[m];
        a.y[ad] = a.first ? v : a.y[ad] + v;
      }
    }
  }
}

}  // namespace cheb
