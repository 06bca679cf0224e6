// Device building blocks for the gfx950 kernels: complex helpers, compile-time
// twiddle constants, register-resident small DFTs and wave-group scans.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cheb {

template <typename T>
struct alignas(2 * sizeof(T)) cplx {
  T x, y;
};

// ---------------------------------------------------------------------------
// Compile-time cos/sin of 2*pi*e/R: octant reduction to [0, pi/4] and a
// Taylor series (14 terms, truncation error far below one ulp on [0, pi/4]).
// Used for the twiddles inside the register DFTs, where every index is a
// compile-time constant after unrolling.
// ---------------------------------------------------------------------------
constexpr double kPi = 3.141592653589793238462643383279502884;

constexpr double ct_sin_red(double x) {
  double x2 = x * x, t = x, s = x;
  for (int i = 1; i <= 14; ++i) {
    t *= -x2 / double((2 * i) * (2 * i + 1));
    s += t;
  }
  return s;
}

constexpr double ct_cos_red(double x) {
  double x2 = x * x, t = 1.0, s = 1.0;
  for (int i = 1; i <= 14; ++i) {
    t *= -x2 / double((2 * i - 1) * (2 * i));
    s += t;
  }
  return s;
}

// returns cos (want_sin = false) or sin (want_sin = true) of 2*pi*e/R
constexpr double ct_trig2pi(long e, long R, bool want_sin) {
  e = ((e % R) + R) % R;
  long num = 8 * e;
  long o = num / R;        // octant 0..7
  long r = num - o * R;    // angle inside the octant = (pi/4) r / R
  double th = (kPi / 4.0) * double(r) / double(R);
  double ph = (kPi / 4.0) * double(R - r) / double(R);  // pi/4 - th
  double c = 0.0, s = 0.0;
  switch (o) {
    case 0: c = ct_cos_red(th); s = ct_sin_red(th); break;
    case 1: c = ct_sin_red(ph); s = ct_cos_red(ph); break;
    case 2: c = -ct_sin_red(th); s = ct_cos_red(th); break;
    case 3: c = -ct_cos_red(ph); s = ct_sin_red(ph); break;
    case 4: c = -ct_cos_red(th); s = -ct_sin_red(th); break;
    case 5: c = -ct_sin_red(ph); s = -ct_cos_red(ph); break;
    case 6: c = ct_sin_red(th); s = -ct_cos_red(th); break;
    default: c = ct_cos_red(ph); s = -ct_sin_red(ph); break;
  }
  return want_sin ? s : c;
}

constexpr double ct_cos2pi(long e, long R) { return ct_trig2pi(e, R, false); }
constexpr double ct_sin2pi(long e, long R) { return ct_trig2pi(e, R, true); }

// ---------------------------------------------------------------------------
// Register DFTs, forward sign: X_k = sum_j x_j exp(-2 pi i j k / R), in place
// on the slots O + S*i (i < R) of two register arrays.  Composite sizes use one
// Cooley-Tukey split R = A*B (input j = B*j1 + j2, output k = k1 + A*k2) with
// compile-time twiddles; outputs are left in digit-reversed slots, output k in
// slot O + S*dft_pos(R, k).  Every index folds to a constant after unrolling.
// ---------------------------------------------------------------------------
constexpr int dft_split(int R) {
  return (R % 4 == 0 && R != 4) ? 4 : (R % 2 == 0 && R != 2) ? 2 : (R % 3 == 0 && R != 3) ? 3 : 0;
}

constexpr int dft_pos(int R, int k) {
  return R <= 4 ? k : (R / dft_split(R)) * dft_pos(dft_split(R), k % dft_split(R)) +
                          dft_pos(R / dft_split(R), k / dft_split(R));
}

// dft_pos as a constant table, so unrolled loops index registers with literals
template <int R>
struct PosTab {
  int v[R];
};
template <int R>
constexpr PosTab<R> make_pos_tab() {
  PosTab<R> t{};
  for (int k = 0; k < R; ++k) t.v[k] = dft_pos(R, k);
  return t;
}

template <int R, int S, int O, typename T>
__device__ __forceinline__ void dft_ip(T* re, T* im);

// twiddle the outputs k1 = K1..A-1 of column J2 by W_R^{J2 k1}
template <int R, int S, int O, int A, int B, int J2, int K1, typename T>
__device__ __forceinline__ void dft_twiddle(T* re, T* im) {
  if constexpr (K1 < A) {
    constexpr int p = O + S * (B * dft_pos(A, K1) + J2);
    constexpr double c = ct_cos2pi(J2 * K1, R);
    constexpr double s = -ct_sin2pi(J2 * K1, R);
    const T xr = re[p], xi = im[p];
    re[p] = xr * T(c) - xi * T(s);
    im[p] = xr * T(s) + xi * T(c);
    dft_twiddle<R, S, O, A, B, J2, K1 + 1, T>(re, im);
  }
}

template <int R, int S, int O, int A, int B, int J2, typename T>
__device__ __forceinline__ void dft_cols(T* re, T* im) {
  if constexpr (J2 < B) {
    dft_ip<A, S * B, O + S * J2, T>(re, im);
    if constexpr (J2 > 0) dft_twiddle<R, S, O, A, B, J2, 1, T>(re, im);
    dft_cols<R, S, O, A, B, J2 + 1, T>(re, im);
  }
}

template <int R, int S, int O, int A, int B, int K1, typename T>
__device__ __forceinline__ void dft_rows(T* re, T* im) {
  if constexpr (K1 < A) {
    dft_ip<B, S, O + S * B * dft_pos(A, K1), T>(re, im);
    dft_rows<R, S, O, A, B, K1 + 1, T>(re, im);
  }
}

template <int R, int S, int O, typename T>
__device__ __forceinline__ void dft_ip(T* re, T* im) {
  if constexpr (R == 1) {
  } else if constexpr (R == 2) {
    const T ar = re[O], ai = im[O];
    re[O] = ar + re[O + S];
    im[O] = ai + im[O + S];
    re[O + S] = ar - re[O + S];
    im[O + S] = ai - im[O + S];
  } else if constexpr (R == 3) {
    const T h = T(0.5);
    const T s3 = T(0.86602540378443864676372317075293618);  // sin(2 pi/3)
    const T sr = re[O + S] + re[O + 2 * S], si = im[O + S] + im[O + 2 * S];
    const T dr = re[O + S] - re[O + 2 * S], di = im[O + S] - im[O + 2 * S];
    const T mr = re[O] - h * sr, mi = im[O] - h * si;
    re[O] = re[O] + sr;
    im[O] = im[O] + si;
    re[O + S] = mr + s3 * di;
    im[O + S] = mi - s3 * dr;
    re[O + 2 * S] = mr - s3 * di;
    im[O + 2 * S] = mi + s3 * dr;
  } else if constexpr (R == 4) {
    const T ar = re[O] + re[O + 2 * S], ai = im[O] + im[O + 2 * S];
    const T br = re[O] - re[O + 2 * S], bi = im[O] - im[O + 2 * S];
    const T cr = re[O + S] + re[O + 3 * S], ci = im[O + S] + im[O + 3 * S];
    const T dr = re[O + S] - re[O + 3 * S], di = im[O + S] - im[O + 3 * S];
    re[O] = ar + cr;
    im[O] = ai + ci;
    re[O + 2 * S] = ar - cr;
    im[O + 2 * S] = ai - ci;
    re[O + S] = br + di;   // X1 = b - i d
    im[O + S] = bi - dr;
    re[O + 3 * S] = br - di;  // X3 = b + i d
    im[O + 3 * S] = bi + dr;
  } else {
    constexpr int A = dft_split(R);
    static_assert(A != 0, "unsupported register DFT size");
    constexpr int B = R / A;
    dft_cols<R, S, O, A, B, 0, T>(re, im);
    dft_rows<R, S, O, A, B, 0, T>(re, im);
  }
}

template <int R>
struct DFT {
  // forward DFT; afterwards output k sits in slot dft_pos(R, k)
  template <typename T>
  __device__ __forceinline__ static void run(T* re, T* im) {
    dft_ip<R, 1, 0, T>(re, im);
  }
};

// Workgroup barrier over LDS only: waits for this thread's LDS accesses, not
// for its global loads in flight (a __syncthreads() fence waits for those too,
// which serialises a prefetch into the next barrier).  For barriers whose only
// purpose is the exchange through LDS.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------------------------
// Four-step split of the even-extension length L = 2N = R1 * R2 used by the
// pencil DCT-I.  Both factors are register DFT sizes; R2 is even.
// ---------------------------------------------------------------------------
struct Split {
  int r1, r2;
};

constexpr Split fft_split(int L) {
  switch (L) {
    case 8: return {2, 4};
    case 16: return {4, 4};
    case 24: return {4, 6};
    case 32: return {4, 8};
    case 48: return {6, 8};
    case 64: return {8, 8};
    case 96: return {8, 12};
    case 128: return {8, 16};
    case 192: return {12, 16};
    case 256: return {16, 16};
    case 384: return {16, 24};
    case 512: return {16, 32};
    case 768: return {24, 32};
    case 1024: return {32, 32};
    default: return {0, 0};
  }
}

// XCD-aware block order: consecutive logical tiles land on the same XCD (the
// hardware deals workgroups round-robin over the 8 XCDs), so tiles that share
// cache lines share an L2.
__device__ __forceinline__ int xcd_swizzle(int bid, int nb) {
  const int x = bid & 7, slot = bid >> 3;
  const int q = nb >> 3, r = nb & 7;
  return x * q + (x < r ? x : r) + slot;
}

// Group-of-G-lanes suffix (exclusive) sum; G divides 64 and groups are aligned.
template <int G, typename T>
__device__ __forceinline__ T group_suffix_excl(T v, int g) {
  T inc = v;
#pragma unroll
  for (int off = 1; off < G; off <<= 1) {
    T o = __shfl_down(inc, off, G);
    if (g + off < G) inc += o;
  }
  return inc - v;
}

template <int G, typename T>
__device__ __forceinline__ T group_prefix_excl(T v, int g) {
  T inc = v;
#pragma unroll
  for (int off = 1; off < G; off <<= 1) {
    T o = __shfl_up(inc, off, G);
    if (g >= off) inc += o;
  }
  return inc - v;
}

template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int off = G >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
  return v;
}

// Matrix-core multiply-accumulate D += A B on one 16x16x4 block per wave.
// Operand layout (both precisions): lane l holds A(l % 16, l / 16) and
// B(l / 16, l % 16); the accumulator holds column l % 16 and four rows given by
// row(l / 16, r).
template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double __attribute__((ext_vector_type(4))) v4;
  __device__ static v4 mac(double a, double b, v4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  // accumulator element r of lane l is row l/16 + 4 r (vector width 1)
  __device__ static int row(int lk, int r) { return lk + 4 * r; }
};
template <>
struct Mfma<float> {
  typedef float __attribute__((ext_vector_type(4))) v4;
  __device__ static v4 mac(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  // accumulator element r of lane l is row 4 (l/16) + r (vector width 4)
  __device__ static int row(int lk, int r) { return 4 * lk + r; }
};

}  // namespace cheb
