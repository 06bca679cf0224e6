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
// Register DFTs, forward sign: X_k = sum_j x_j exp(-2 pi i j k / R).
// Composite sizes use one Cooley-Tukey split R = A*B (input j = B*j1 + j2,
// output k = k1 + A*k2) with compile-time twiddles.
// ---------------------------------------------------------------------------
constexpr int dft_split(int R) {
  return (R % 4 == 0 && R != 4) ? 4 : (R % 2 == 0 && R != 2) ? 2 : (R % 3 == 0 && R != 3) ? 3 : 0;
}

template <int R>
struct DFT {
  template <typename T>
  __device__ __forceinline__ static void run(T* re, T* im) {
    constexpr int A = dft_split(R);
    static_assert(A != 0, "unsupported register DFT size");
    constexpr int B = R / A;
    T zr[A][B], zi[A][B];
#pragma unroll
    for (int j2 = 0; j2 < B; ++j2) {
      T ar[A], ai[A];
#pragma unroll
      for (int j1 = 0; j1 < A; ++j1) {
        ar[j1] = re[B * j1 + j2];
        ai[j1] = im[B * j1 + j2];
      }
      DFT<A>::run(ar, ai);
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1) {
        const T c = T(ct_cos2pi(j2 * k1, R));
        const T s = T(-ct_sin2pi(j2 * k1, R));
        if (j2 * k1 == 0) {
          zr[k1][j2] = ar[k1];
          zi[k1][j2] = ai[k1];
        } else {
          zr[k1][j2] = ar[k1] * c - ai[k1] * s;
          zi[k1][j2] = ar[k1] * s + ai[k1] * c;
        }
      }
    }
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
      DFT<B>::run(zr[k1], zi[k1]);
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) {
        re[k1 + A * k2] = zr[k1][k2];
        im[k1 + A * k2] = zi[k1][k2];
      }
    }
  }
};

template <>
struct DFT<1> {
  template <typename T>
  __device__ __forceinline__ static void run(T*, T*) {}
};

template <>
struct DFT<2> {
  template <typename T>
  __device__ __forceinline__ static void run(T* re, T* im) {
    T ar = re[0], ai = im[0];
    re[0] = ar + re[1];
    im[0] = ai + im[1];
    re[1] = ar - re[1];
    im[1] = ai - im[1];
  }
};

template <>
struct DFT<3> {
  template <typename T>
  __device__ __forceinline__ static void run(T* re, T* im) {
    const T h = T(0.5);
    const T s3 = T(0.86602540378443864676372317075293618);  // sin(2 pi/3)
    T sr = re[1] + re[2], si = im[1] + im[2];
    T dr = re[1] - re[2], di = im[1] - im[2];
    T mr = re[0] - h * sr, mi = im[0] - h * si;
    re[0] = re[0] + sr;
    im[0] = im[0] + si;
    // X1 = m - i s3 d, X2 = m + i s3 d
    re[1] = mr + s3 * di;
    im[1] = mi - s3 * dr;
    re[2] = mr - s3 * di;
    im[2] = mi + s3 * dr;
  }
};

template <>
struct DFT<4> {
  template <typename T>
  __device__ __forceinline__ static void run(T* re, T* im) {
    T ar = re[0] + re[2], ai = im[0] + im[2];
    T br = re[0] - re[2], bi = im[0] - im[2];
    T cr = re[1] + re[3], ci = im[1] + im[3];
    T dr = re[1] - re[3], di = im[1] - im[3];
    re[0] = ar + cr;
    im[0] = ai + ci;
    re[2] = ar - cr;
    im[2] = ai - ci;
    // X1 = b - i d, X3 = b + i d
    re[1] = br + di;
    im[1] = bi - dr;
    re[3] = br - di;
    im[3] = bi + dr;
  }
};

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

}  // namespace cheb
