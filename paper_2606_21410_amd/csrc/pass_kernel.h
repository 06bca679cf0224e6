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
//
// Occupancy: a tile is one wave.  The exchange buffer aliases the pencil
// buffer (every thread moves its items into registers, then a barrier, then
// the writes), which roughly halves the LDS per pencil; strides are odd in
// 16-byte units so the b128 exchange accesses are free of bank conflicts.
#pragma once

#include "dev_common.h"
#include "pencil.h"

namespace cheb {

// MODE_DERIV_ACC: y += D_a (K * V) on the interior nodes of interior-transverse
// pencils, V the homogeneous lift of u's interior values, formed in the pencil
// as in MODE_REDUCED (the Newton Jacobian's k'(T) term, K standing for
// k'(T) D_a T)
enum PassMode { MODE_FULL = 0, MODE_REDUCED = 1, MODE_TRANSPOSE = 2, MODE_DERIV = 3, MODE_DERIV_T = 4,
                MODE_DERIV_ACC = 5 };

template <typename T>
struct PassArgs {
  const int* gate;  // null, or a device flag: the pass does nothing while it reads 0
  const T* u;
  const T* K;
  T* y;
  const T* drow0;  // row 0 of the ascending, scaled differentiation matrix (n entries)
  const T* drowN;  // row N
  const T* twg;    // W_2N^j, j < 2N, interleaved (re, im)
  int n[3];
  int axis;
  int N;      // n[axis] - 1
  int first;  // this pass initialises every row it owns ('='); later passes accumulate
  int bcmask; // bit f set when face f is Neumann
  T cscale;   // -1 / (N * L_axis)
  T m00, m0N, mN0, mNN;  // end-value block of the boundary rows (corner entries, Robin-shifted)
  T slo, shi;            // Robin coefficients of the axis' lo and hi faces (FULL rows)
  // per-node Robin coefficients (packed faces) or null; rlo / rhi: offsets of
  // the axis' lo and hi faces, whose entries follow the pencil numbering
  const T* rnode;
  int rlo, rhi;
  int npencils;
};

// ---------------------------------------------------------------------------
// Tile shape per transform size (NC = 0: generic size, direct DCT)
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int pass_threads(int NC) { return 64; }
__host__ __device__ constexpr int pass_pencils(int NC) {
  return NC == 0 ? 8 : NC <= 16 ? 16 : NC <= 48 ? 8 : NC <= 64 ? 4 : NC <= 128 ? 8 : 4;
}
__host__ __device__ constexpr int exch_stride(int r2) { return (r2 / 2 + 1) | 1; }

struct PassLayout {
  int buf_off, tw_off, tmp_off, ends_off, base_off, flags_off, bytes, svs;
};

// LDS layout (bytes) of one tile.
template <typename T>
__host__ __device__ constexpr PassLayout pass_layout(int NC, int Nrt) {
  const int N = NC > 0 ? NC : Nrt;
  const int P = pass_pencils(NC);
  const int n = N + 1;
  const int svs = n + 1;
  PassLayout l{0, 0, 0, 0, 0, 0, 0, svs};
  int off = 0;
  const int sv_bytes = P * svs * (int)sizeof(T);
  if (NC > 0) {
    const Split sp = fft_split(2 * N);
    const int e_bytes = (P / 2) * sp.r1 * exch_stride(sp.r2) * 2 * (int)sizeof(T);
    l.buf_off = 0;
    off = ((e_bytes > sv_bytes ? e_bytes : sv_bytes) + 15) & ~15;
    l.tw_off = off;
    off += 2 * N * 2 * (int)sizeof(T);
    l.tmp_off = off;
  } else {
    l.buf_off = 0;
    off = (sv_bytes + 15) & ~15;
    l.tmp_off = off;
    off += (sv_bytes + 15) & ~15;
    l.tw_off = off;  // cos(pi j / N), j < 2N
    off += 2 * N * (int)sizeof(T);
  }
  off = (off + 15) & ~15;
  l.ends_off = off;
  off += 4 * P * (int)sizeof(T);
  off = (off + 15) & ~15;
  l.base_off = off;
  off += P * 4;
  l.flags_off = off;
  off += P * 4;
  l.bytes = (off + 15) & ~15;
  return l;
}

// ---------------------------------------------------------------------------
// DCT-I of all pencils of the tile, in place in sv (pencil stride N+2); the
// exchange buffer E aliases sv.
// ---------------------------------------------------------------------------
template <typename T, int NC, int P, int NT>
__device__ __forceinline__ void dct_tile_fast(T* sv, const cplx<T>* tw, int tid) {
  constexpr int N = NC, L = 2 * N, SVS = N + 2;
  constexpr Split sp = fft_split(L);
  constexpr int R1 = sp.r1, R2 = sp.r2, H = R2 / 2 + 1, EH = exch_stride(R2), Q = P / 2;
  constexpr int IT1 = (Q * H + NT - 1) / NT, IT2 = (Q * R1 + NT - 1) / NT;
  static_assert(R1 > 0 && R2 % 2 == 0, "transform size not supported");
  constexpr PosTab<R1> pos1 = make_pos_tab<R1>();
  constexpr PosTab<R2> pos2 = make_pos_tab<R2>();
  cplx<T>* E = reinterpret_cast<cplx<T>*>(sv);
  // stage 1: columns n2 = 0..R2/2, DFT over n1, twiddle W_L^{n2 k1}
  T re1[IT1][R1], im1[IT1][R1];
#pragma unroll
  for (int it = 0; it < IT1; ++it) {
    const int w = tid + it * NT;
    if (w < Q * H) {
      const int q = w / H, n2 = w - q * H;
      const T* a = sv + (2 * q) * SVS;
      const T* b = a + SVS;
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) {
        const int m = R2 * n1 + n2;
        const int s = m <= N ? m : L - m;
        re1[it][n1] = a[s];
        im1[it][n1] = b[s];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IT1; ++it) {
    const int w = tid + it * NT;
    if (w < Q * H) {
      const int q = w / H, n2 = w - q * H;
      DFT<R1>::run(re1[it], im1[it]);
      cplx<T>* e = E + (q * R1) * EH + n2;
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) {
        const cplx<T> t = tw[n2 * k1];
        cplx<T> v;
        const T xr = re1[it][pos1.v[k1]], xi = im1[it][pos1.v[k1]];
        v.x = xr * t.x - xi * t.y;
        v.y = xr * t.y + xi * t.x;
        e[k1 * EH] = v;
      }
    }
  }
  __syncthreads();
  // stage 2: rows k1, DFT over n2 (columns > R2/2 from the mirrored row)
  T re2[IT2][R2], im2[IT2][R2];
#pragma unroll
  for (int it = 0; it < IT2; ++it) {
    const int w = tid + it * NT;
    if (w < Q * R1) {
      const int q = w / R1, k1 = w - q * R1;
      const int k1p = k1 == 0 ? 0 : R1 - k1;
      const cplx<T>* e = E + (q * R1) * EH;
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) {
        if (n2 <= R2 / 2) {
          const cplx<T> v = e[k1 * EH + n2];
          re2[it][n2] = v.x;
          im2[it][n2] = v.y;
        } else {
          const cplx<T> v = e[k1p * EH + (R2 - n2)];
          re2[it][n2] = v.x;
          im2[it][n2] = v.y;
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IT2; ++it) {
    const int w = tid + it * NT;
    if (w < Q * R1) {
      const int q = w / R1, k1 = w - q * R1;
      if (k1 != 0) {
#pragma unroll
        for (int n2 = R2 / 2 + 1; n2 < R2; ++n2) {
          const T c = T(ct_cos2pi(n2, R2)), s = T(-ct_sin2pi(n2, R2));
          const T vr = re2[it][n2] * c - im2[it][n2] * s;
          const T vi = re2[it][n2] * s + im2[it][n2] * c;
          re2[it][n2] = vr;
          im2[it][n2] = vi;
        }
      }
      DFT<R2>::run(re2[it], im2[it]);
      T* a = sv + (2 * q) * SVS;
      T* b = a + SVS;
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) {
        const int k = k1 + R1 * k2;
        if (k <= N) {
          a[k] = re2[it][pos2.v[k2]];
          b[k] = im2[it][pos2.v[k2]];
        }
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
// Coefficient-space recurrences on one pencil, G lanes per pencil, each lane a
// contiguous chunk of CH coefficients (CH even; compile-time for fast sizes).
// ---------------------------------------------------------------------------
template <typename T, int G, int CH>
__device__ __forceinline__ void recur_forward(T* pen, int N, T c, int g) {
  const int n = N + 1;
  const int j0 = g * CH;
  T w[CH];
  T t0 = T(0), t1 = T(0);
#pragma unroll
  for (int i = 0; i < CH; ++i) {
    const int j = j0 + i;
    T v = T(0);
    if (j < n) v = pen[j] * T(j) * ((j == 0 || j == N) ? T(1) : T(2));
    w[i] = v;
    if (i & 1) t1 += v; else t0 += v;  // j0 even: parity of j = parity of i
  }
  T r0 = group_suffix_excl<G>(t0, g);
  T r1 = group_suffix_excl<G>(t1, g);
#pragma unroll
  for (int i = CH - 1; i >= 0; --i) {
    const int j = j0 + i;
    const T beta = (i & 1) ? r0 : r1;  // sum of w_l, l > j, l of the other parity
    if (j < n) pen[j] = c * beta;
    if (i & 1) r1 += w[i]; else r0 += w[i];
  }
}

template <typename T, int G, int CH>
__device__ __forceinline__ void recur_transpose(T* pen, int N, T c, int g) {
  const int n = N + 1;
  const int j0 = g * CH;
  T t[CH];
  T t0 = T(0), t1 = T(0);
#pragma unroll
  for (int i = 0; i < CH; ++i) {
    const int j = j0 + i;
    T v = T(0);
    if (j < n) v = pen[j] * ((j == 0 || j == N) ? T(1) : T(2));
    t[i] = v;
    if (i & 1) t1 += v; else t0 += v;
  }
  T r0 = group_prefix_excl<G>(t0, g);
  T r1 = group_prefix_excl<G>(t1, g);
#pragma unroll
  for (int i = 0; i < CH; ++i) {
    const int j = j0 + i;
    const T rho = (i & 1) ? r0 : r1;  // sum of t_k, k < j, k of the other parity
    if (j < n) pen[j] = c * T(j) * rho;
    if (i & 1) r1 += t[i]; else r0 += t[i];
  }
}

// runtime-size variants (generic path)
template <typename T, int G>
__device__ __forceinline__ void recur_forward_rt(T* pen, int N, T c, int g) {
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
    const T beta = (j & 1) ? r0 : r1;
    pen[j] = c * beta;
    if (j & 1) r1 += w; else r0 += w;
  }
}

template <typename T, int G>
__device__ __forceinline__ void recur_transpose_rt(T* pen, int N, T c, int g) {
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
    const T rho = (j & 1) ? r0 : r1;
    pen[j] = c * T(j) * rho;
    if (j & 1) r1 += t; else r0 += t;
  }
}

template <typename T, int NC, int P, int NT>
__device__ __forceinline__ void pass_dct(T* sv, T* tmp, const cplx<T>* tw, const T* ctab, int N, int tid) {
  if constexpr (NC > 0) dct_tile_fast<T, NC, P, NT>(sv, tw, tid);
  else dct_tile_direct<T, P, NT>(sv, tmp, ctab, N, tid);
}

template <typename T, int NC, int MODE, int G, int CH>
__device__ __forceinline__ void pass_recur(T* pen, int N, T c, int g) {
  constexpr bool tr = (MODE == MODE_TRANSPOSE || MODE == MODE_DERIV_T);
  if constexpr (NC > 0) {
    if constexpr (tr) recur_transpose<T, G, CH>(pen, N, c, g);
    else recur_forward<T, G, CH>(pen, N, c, g);
  } else {
    if constexpr (tr) recur_transpose_rt<T, G>(pen, N, c, g);
    else recur_forward_rt<T, G>(pen, N, c, g);
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// The pass kernel
// ---------------------------------------------------------------------------
// element e of a tile -> (pencil slot pl, node m); pencils are contiguous in
// memory along z, interleaved (slot fastest) along x and y.  (A macro: passing
// pl and m by reference to a helper made the compiler keep them in scratch.)
#define TILE_MAP(e, pl, m)  \
  if (contig) {             \
    pl = (e) / n;           \
    m = (e) - pl * n;       \
  } else {                  \
    m = (e) / P;            \
    pl = (e) - m * P;       \
  }

template <typename T, int NC, int MODE>
__global__ __launch_bounds__(pass_threads(NC)) void k_axis_pass(PassArgs<T> a) {
  if (a.gate && !*a.gate) return;
  constexpr int P = pass_pencils(NC);
  constexpr int NT = pass_threads(NC);
  constexpr int G = NT / P;
  constexpr int CH = NC > 0 ? ((((NC + 1) + G - 1) / G + 1) & ~1) : 0;
  static_assert(NT % P == 0 && 64 % G == 0, "bad tile shape");
  // elements of the tile per thread, and whether one register chunk holds them
  constexpr int EPT = NC > 0 ? (P * (NC + 1) + NT - 1) / NT : 8;
  constexpr int CHK = EPT < 24 ? EPT : 24;
  constexpr bool ONE = NC > 0 && CHK * NT >= P * (NC + 1);
  constexpr bool NEEDK = (MODE != MODE_DERIV && MODE != MODE_DERIV_T && MODE != MODE_DERIV_ACC);
  constexpr bool ACC = (MODE == MODE_FULL || MODE == MODE_REDUCED || MODE == MODE_TRANSPOSE ||
                        MODE == MODE_DERIV_ACC);
  // K held in registers through the first derivative: up to 12 elements per
  // thread, and up to 18 for FP64 at N >= 192 (N = 192, 256: the apply 2.7% and
  // 4.5% faster; at N = 128 the registers cost occupancy and the FP64 apply
  // slowed by a third, at N = 256 in FP32 by a quarter)
  constexpr bool PRE_K = ONE && NEEDK && CHK <= ((sizeof(T) == 8 && NC >= 192) ? 18 : 12);
  constexpr bool PRE_Y = ONE && ACC && CHK <= 12;
  extern __shared__ __align__(16) unsigned char smem[];
  const int N = NC > 0 ? NC : a.N;
  const int n = N + 1;
  const PassLayout lay = pass_layout<T>(NC, N);
  const int SVS = lay.svs;
  T* sv = (T*)(smem + lay.buf_off);
  T* ends = (T*)(smem + lay.ends_off);
  int* base = (int*)(smem + lay.base_off);
  int* flags = (int*)(smem + lay.flags_off);
  cplx<T>* tw = (cplx<T>*)(smem + lay.tw_off);
  T* tmp = (T*)(smem + lay.tmp_off);
  T* ctab = (T*)(smem + lay.tw_off);

  const int tid = threadIdx.x;
  const int tile = xcd_swizzle(blockIdx.x, gridDim.x);
  const int p0 = tile * P;
  const int axis = a.axis;
  const int n1 = a.n[1], n2 = a.n[2];
  const int stride = axis == 2 ? 1 : axis == 1 ? n2 : n1 * n2;
  const bool contig = axis == 2;
  const int TOT = P * n;

  // pencil classification (computed redundantly per lane, kept in LDS for the loops)
  int my_fl = 0, my_base = 0;
  if (tid < P) {
    long long b = 0;
    my_fl = pencil_flags(axis, p0 + tid, a.npencils, a.n[0], a.n[1], a.n[2], a.bcmask, &b);
    my_base = (int)b;
    flags[tid] = my_fl;
    base[tid] = my_base;
  }
  // twiddles W_L^j from the plan's table (fast path) or cos(pi j/N) (direct path)
  if (NC > 0) {
    const cplx<T>* twg = reinterpret_cast<const cplx<T>*>(a.twg);
    for (int j = tid; j < 2 * N; j += NT) tw[j] = twg[j];
  } else {
    for (int j = tid; j < 2 * N; j += NT) ctab[j] = T(cospi(double(j) / double(N)));
  }
  __syncthreads();


  // Global loads: with ONE, u, K (and y when accumulating with few elements)
  // are all requested up front so the tile waits for memory once.
  T kv[PRE_K ? CHK : 1];
  T yv[PRE_Y ? CHK : 1];
  for (int e0 = 0; e0 < TOT; e0 += NT * CHK) {
    T v[CHK];
#pragma unroll
    for (int c = 0; c < CHK; ++c) {
      const int e = e0 + c * NT + tid;
      v[c] = T(0);
      if (PRE_K) kv[PRE_K ? c : 0] = T(0);
      if (PRE_Y) yv[c] = T(0);
      if (e < TOT) {
        int pl, m;
        TILE_MAP(e, pl, m);
        const int fl = flags[pl];
        if (fl & PF_VALID) {
          const int ad = base[pl] + m * stride;
          const bool ld = (MODE == MODE_FULL || MODE == MODE_DERIV || MODE == MODE_DERIV_T) || (fl & PF_TIN);
          if (MODE == MODE_DERIV_ACC) {
            // interior values times K; the end values come from the lift below
            if ((fl & PF_TIN) && m != 0 && m != N) v[c] = a.u[ad] * a.K[ad];
          } else if (ld) {
            v[c] = a.u[ad];
          }
          if (PRE_K) kv[PRE_K ? c : 0] = a.K[ad];
          if (PRE_Y && !a.first && (fl & PF_TIN) && m != 0 && m != N) yv[c] = a.y[ad];
        }
      }
    }
#pragma unroll
    for (int c = 0; c < CHK; ++c) {
      const int e = e0 + c * NT + tid;
      if (e < TOT) {
        int pl, m;
        TILE_MAP(e, pl, m);
        T x = v[c];
        if (MODE == MODE_DERIV_T && m != 0 && m != N) x *= T(0.5);
        if (MODE == MODE_REDUCED || MODE == MODE_TRANSPOSE) {
          if (m == 0 || m == N) x = T(0);
          else if (MODE == MODE_TRANSPOSE) x *= T(0.5);
        }
        if (MODE == MODE_FULL) {
          if (m == 0) ends[4 * pl + 0] = x;
          if (m == N) ends[4 * pl + 1] = x;
        }
        sv[pl * SVS + m] = x;
      }
    }
  }
  __syncthreads();

  const int pp = tid / G, g = tid - pp * G;
  T* pen = sv + pp * SVS;

  if (MODE == MODE_REDUCED || MODE == MODE_DERIV_ACC) {
    // homogeneous lift of the pencil's end values (Neumann rows, Section 2.3.1);
    // MODE_DERIV_ACC holds K * u in the tile, so its row sums read u itself
    T s0 = T(0), sN = T(0);
    const int pb = base[pp];
    for (int m = 1 + g; m < N; m += G) {
      const T v = MODE == MODE_DERIV_ACC ? ((flags[pp] & PF_TIN) ? a.u[pb + m * stride] : T(0)) : pen[m];
      s0 += a.drow0[m] * v;
      sN += a.drowN[m] * v;
    }
    s0 = group_sum<G>(s0);
    sN = group_sum<G>(sN);
    const int fl = flags[pp];
    if (g == 0 && (fl & PF_TIN)) {
      const bool nlo = (a.bcmask >> (2 * axis)) & 1, nhi = (a.bcmask >> (2 * axis + 1)) & 1;
      T m00 = a.m00, mNN = a.mNN;
      if (a.rnode) {
        m00 -= a.rnode[a.rlo + p0 + pp];
        mNN += a.rnode[a.rhi + p0 + pp];
      }
      T u0 = T(0), uN = T(0);
      if (nlo && nhi) {
        const T det = m00 * mNN - a.m0N * a.mN0;
        u0 = (-s0 * mNN + sN * a.m0N) / det;
        uN = (-sN * m00 + s0 * a.mN0) / det;
      } else if (nlo) {
        u0 = -s0 / m00;
      } else if (nhi) {
        uN = -sN / mNN;
      }
      if (MODE == MODE_DERIV_ACC) {
        u0 *= a.K[pb];
        uN *= a.K[pb + N * stride];
      }
      pen[0] = u0;
      pen[N] = uN;
    }
    __syncthreads();
  }

  // first derivative (or its transpose)
  pass_dct<T, NC, P, NT>(sv, tmp, tw, ctab, N, tid);
  pass_recur<T, NC, MODE, G, CH>(pen, N, a.cscale, g);
  pass_dct<T, NC, P, NT>(sv, tmp, tw, ctab, N, tid);

  if (NEEDK) {
    // pointwise flux K * D_a u (boundary nodes included)
    for (int e0 = 0; e0 < TOT; e0 += NT * CHK) {
      T k2[PRE_K ? 1 : CHK];
      if (!PRE_K) {
#pragma unroll
        for (int c = 0; c < CHK; ++c) {
          const int e = e0 + c * NT + tid;
          k2[PRE_K ? 0 : c] = T(0);
          if (e < TOT) {
            int pl, m;
            TILE_MAP(e, pl, m);
            if (flags[pl] & PF_VALID) k2[PRE_K ? 0 : c] = a.K[base[pl] + m * stride];
          }
        }
      }
#pragma unroll
      for (int c = 0; c < CHK; ++c) {
        const int e = e0 + c * NT + tid;
        if (e < TOT) {
          int pl, m;
          TILE_MAP(e, pl, m);
          const T x = sv[pl * SVS + m];
          if (MODE == MODE_FULL) {
            if (m == 0) ends[4 * pl + 2] = x;
            if (m == N) ends[4 * pl + 3] = x;
          }
          sv[pl * SVS + m] = x * (PRE_K ? kv[PRE_K ? c : 0] : k2[PRE_K ? 0 : c]);
        }
      }
    }
    __syncthreads();
    // divergence part
    pass_dct<T, NC, P, NT>(sv, tmp, tw, ctab, N, tid);
    pass_recur<T, NC, MODE, G, CH>(pen, N, a.cscale, g);
    pass_dct<T, NC, P, NT>(sv, tmp, tw, ctab, N, tid);
  }

  if (MODE == MODE_TRANSPOSE) {
    // transposed lift: mu = M^{-T} [z_0, z_N]; interior -= mu0 D_{0,:} + muN D_{N,:}
    if (g == 0) {
      const bool nlo = (a.bcmask >> (2 * axis)) & 1, nhi = (a.bcmask >> (2 * axis + 1)) & 1;
      const T z0 = pen[0], zN = pen[N];
      T m00 = a.m00, mNN = a.mNN;
      if (a.rnode && (flags[pp] & PF_VALID)) {
        m00 -= a.rnode[a.rlo + p0 + pp];
        mNN += a.rnode[a.rhi + p0 + pp];
      }
      T mu0 = T(0), muN = T(0);
      if (nlo && nhi) {
        const T det = m00 * mNN - a.m0N * a.mN0;
        mu0 = (z0 * mNN - zN * a.mN0) / det;
        muN = (zN * m00 - z0 * a.m0N) / det;
      } else if (nlo) {
        mu0 = z0 / m00;
      } else if (nhi) {
        muN = zN / mNN;
      }
      ends[4 * pp + 0] = mu0;
      ends[4 * pp + 1] = muN;
    }
    __syncthreads();
  }

  // store (accumulating passes without prefetched y load their chunk first)
  for (int e0 = 0; e0 < TOT; e0 += NT * CHK) {
    T y2[PRE_Y ? 1 : CHK];
    if (!PRE_Y) {
#pragma unroll
      for (int c = 0; c < CHK; ++c) {
        const int e = e0 + c * NT + tid;
        y2[PRE_Y ? 0 : c] = T(0);
        if (ACC && !a.first && e < TOT) {
          int pl, m;
          TILE_MAP(e, pl, m);
          const int fl = flags[pl];
          if ((fl & PF_VALID) && (fl & PF_TIN) && m != 0 && m != N) y2[PRE_Y ? 0 : c] = a.y[base[pl] + m * stride];
        }
      }
    }
#pragma unroll
    for (int c = 0; c < CHK; ++c) {
      const int e = e0 + c * NT + tid;
      if (e >= TOT) continue;
      int pl, m;
      TILE_MAP(e, pl, m);
      const int fl = flags[pl];
      if (!(fl & PF_VALID)) continue;
      const int ad = base[pl] + m * stride;
      const T yold = PRE_Y ? yv[PRE_Y ? c : 0] : y2[PRE_Y ? 0 : c];
      T x = sv[pl * SVS + m];
      const bool isend = (m == 0 || m == N);
      if (MODE == MODE_DERIV) {
        a.y[ad] = x;
      } else if (MODE == MODE_DERIV_T) {
        a.y[ad] = isend ? x : T(2) * x;
      } else if (MODE == MODE_DERIV_ACC) {
        if ((fl & PF_TIN) && !isend) a.y[ad] = a.first ? x : yold + x;
      } else if (MODE == MODE_FULL) {
        if (!isend) {
          if (fl & PF_TIN) a.y[ad] = a.first ? x : yold + x;
        } else {
          const bool own = (m == 0) ? (fl & PF_OWN_LO) : (fl & PF_OWN_HI);
          if (own) {
            const int bct = (a.bcmask >> (2 * axis + (m == 0 ? 0 : 1))) & 1;
            T r;
            if (bct == 0) {
              r = ends[4 * pl + (m == 0 ? 0 : 1)];
            } else {
              const T sig = (m == 0 ? a.slo : a.shi) + (a.rnode ? a.rnode[(m == 0 ? a.rlo : a.rhi) + p0 + pl] : T(0));
              r = (m == 0) ? sig * ends[4 * pl + 0] - ends[4 * pl + 2] : ends[4 * pl + 3] + sig * ends[4 * pl + 1];
            }
            a.y[ad] = r;
          }
        }
      } else {
        if (!(fl & PF_TIN) || isend) {
          if (a.first) a.y[ad] = T(0);
        } else {
          if (MODE == MODE_TRANSPOSE)
            x = T(2) * x - ends[4 * pl + 0] * a.drow0[m] - ends[4 * pl + 1] * a.drowN[m];
          a.y[ad] = a.first ? x : yold + x;
        }
      }
    }
  }
  (void)my_fl;
  (void)my_base;
}

#undef TILE_MAP

}  // namespace cheb
