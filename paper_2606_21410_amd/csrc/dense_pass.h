// Matrix-core route of one axis pass of the reduced operator and of its
// transpose, for axes with N <= 128.
//
// Along axis a the pass computes, for every pencil whose two transverse indices
// are interior,
//   reduced:    y_int (+)= [ D (K .* (D L u_int)) ]_int
//   transpose:  y_int (+)= L^T D^T (K .* (D^T w)),   w zero at the two ends,
// with D the collocation derivative of the axis (Section 2.2) and L the
// homogeneous lift of the pencil's end values from the face rows (Section
// 2.3.1).  For N <= 128 the derivative of a tile of pencils is a small dense
// contraction, so it runs as a batched GEMM on the matrix cores: a tile of C
// pencils is staged in LDS as an n x C matrix and multiplied by D twice, with
// the pointwise flux in between.
//
// Even-odd split: D (and D^T) is centro-antisymmetric, M[N-i][N-j] = -M[i][j],
// so with o_j = u_j - u_{N-j} and e_j = u_j + u_{N-j}
//   (Mu)_i = s_i + d_i,  (Mu)_{N-i} = s_i - d_i,   i <= N/2,
//   s_i = sum_{j < KO} Ao[i][j] o_j,   d_i = sum_{j < KE} Ae[i][j] e_j,
//   Ao[i][j] = (M[i][j] - M[i][N-j]) / 2,  Ae[i][j] = (M[i][j] + M[i][N-j]) / 2
// (Ae[i][N/2] = M[i][N/2] / 2 for even N, where e_{N/2} = 2 u_{N/2}), which
// halves the multiply-adds of the dense product.
#pragma once

#include "dev_common.h"
#include "pencil.h"

namespace cheb {

enum DenseMode { DENSE_REDUCED = 0, DENSE_TRANSPOSE = 1 };

// Compile-time shape of the split product for one N (also used by the host
// code that writes the fragment tables and sizes the LDS).
struct DenseDims {
  int N, HALF, KO, KE, KO4, KE4, R, RM, MT, WC, NW, C, OFF_E, OFF_MID, TAB;
  bool EVEN, MIDV;
};

__host__ __device__ constexpr DenseDims dense_dims(int N) {
  DenseDims d{};
  d.N = N;
  d.HALF = N / 2;
  d.EVEN = (N % 2) == 0;
  d.KO = d.EVEN ? d.HALF : d.HALF + 1;  // odd-part columns j < KO (o_{N/2} = 0)
  d.KE = d.HALF + 1;                     // even-part columns j <= N/2
  d.KO4 = (d.KO + 3) / 4;
  d.KE4 = (d.KE + 3) / 4;
  d.R = d.HALF + 1;                      // output row pairs (i, N-i), i <= N/2
  d.MIDV = d.EVEN && (d.R % 16 == 1);    // a lone middle row goes to the vector ALUs
  d.RM = d.MIDV ? d.R - 1 : d.R;         // rows on the matrix cores
  d.MT = (d.RM + 15) / 16;               // 16-row blocks, one per wave
  d.WC = d.MT == 3 ? 2 : 8 / d.MT;       // 16-column groups per workgroup
  d.NW = d.MT * d.WC;                    // waves per workgroup (8, or 6 for MT = 3)
  d.C = 16 * d.WC;                       // pencils per tile
  // fragment table: [mt][ks][lane] for Ao, then Ae, then the middle row of Ao
  d.OFF_E = d.MT * d.KO4 * 64;
  d.OFF_MID = d.OFF_E + d.MT * d.KE4 * 64;
  d.TAB = d.OFF_MID + d.KO4 * 4;
  return d;
}

__host__ __device__ constexpr bool dense_supported(int N) {
  return N == 16 || N == 32 || N == 48 || N == 64 || N == 96 || N == 128;
}

__host__ __device__ constexpr int pow2_floor(int x) {
  int p = 1;
  while (2 * p <= x) p *= 2;
  return p;
}

// LDS carve of one workgroup (bytes): fragment table, tile, face rows, the
// transposed-lift multipliers, column bookkeeping
template <typename T>
__host__ __device__ constexpr int dense_lds_bytes(int N) {
  const DenseDims d = dense_dims(N);
  const int n = N + 1, SC = d.C + 1;
  return (d.TAB + n * SC + 2 * n + 2 * d.C) * (int)sizeof(T) + 2 * d.C * (int)sizeof(int);
}

template <typename T>
struct DenseArgs {
  const T* u;
  const T* K;
  T* y;
  const T* tab;    // fragment table of D (reduced) or D^T (transpose)
  const T* drow0;  // face rows D[0][:], D[N][:] for the lift
  const T* drowN;
  T* sink;         // one word that stores of off-tile elements go to
  int n[3];
  int axis, first, bcmask, npencils;
  T m00, m0N, mN0, mNN;
};

// tile element e -> (node j along the pencil, column c): pencil-contiguous for
// the unit-stride axis, column-contiguous otherwise, so global accesses coalesce
#define DENSE_MAP(e, j, c)   \
  do {                       \
    if (contig) {            \
      c = (e) / n;           \
      j = (e) - c * n;       \
    } else {                 \
      j = (e) / C;           \
      c = (e) - j * C;       \
    }                        \
  } while (0)

// ACCO/ACCE = split products of the LDS tile (B operand) with this wave's A
// fragments (from the LDS table).  Rows j > N/2 of the last k-step meet zero
// table entries.
#define DENSE_GEMM(ACCO, ACCE)                                                 \
  do {                                                                         \
    ACCO = V4{0, 0, 0, 0};                                                     \
    ACCE = V4{0, 0, 0, 0};                                                     \
    _Pragma("unroll") for (int ks = 0; ks < S.KE4; ++ks) {                     \
      const int j = 4 * ks + lk;                                               \
      const T x0 = U[j * SC + col], x1 = U[(N - j) * SC + col];                \
      if (ks < S.KO4) ACCO = Mfma<T>::mac(Ao[ks * 64], x0 - x1, ACCO);         \
      ACCE = Mfma<T>::mac(Ae[ks * 64], x0 + x1, ACCE);                         \
    }                                                                          \
  } while (0)

// middle row N/2 (odd part only) when it does not fill a 16-row block
#define DENSE_MID(OUT)                                                                 \
  do {                                                                                 \
    OUT = T(0);                                                                        \
    if (S.MIDV) {                                                                      \
      if (lc < C)                                                                      \
        for (int j = lg; j < S.KO; j += LPC) OUT += amid[j] * (U[j * SC + lc] - U[(N - j) * SC + lc]); \
      OUT = group_sum<LPC>(OUT);                                                       \
    }                                                                                  \
  } while (0)

// accumulators -> LDS tile rows i and N-i
#define DENSE_EPI(ACCO, ACCE, MIDVAL)                                      \
  do {                                                                     \
    _Pragma("unroll") for (int r = 0; r < 4; ++r) {                        \
      const int i = 16 * mt + Mfma<T>::row(lk, r);                         \
      if (i < S.RM) {                                                      \
        const T o = ACCO[r], e = ACCE[r];                                  \
        if (2 * i == N) {                                                  \
          U[i * SC + col] = o;                                             \
        } else {                                                           \
          U[i * SC + col] = o + e;                                         \
          U[(N - i) * SC + col] = o - e;                                   \
        }                                                                  \
      }                                                                    \
    }                                                                      \
    if (S.MIDV && lc < C && lg == 0) U[S.HALF * SC + lc] = MIDVAL;         \
  } while (0)

// column bookkeeping of tile TILE into slot SLOT: linear offset of each
// interior-transverse pencil's first node, -1 past the last pencil
#define DENSE_COLS(SLOT, TILE)                                             \
  do {                                                                     \
    if (tid < C) {                                                         \
      const int q_ = (TILE) * C + tid;                                     \
      int b_ = -1;                                                         \
      if (q_ < npen) {                                                     \
        const int ia_ = 1 + q_ / nbi, ib_ = 1 + (q_ - (q_ / nbi) * nbi);   \
        b_ = axis == 2 ? (ia_ * n1 + ib_) * n2 : axis == 1 ? ia_ * n1 * n2 + ib_ : ia_ * n2 + ib_; \
      }                                                                    \
      cbase[SLOT][tid] = b_;                                               \
    }                                                                      \
  } while (0)

// global -> registers: u (interior nodes) and K of the tile in slot SLOT.
// Every load is issued (off-tile elements read node 0 and are discarded), so
// the number of outstanding loads is static and the compiler's waits stay exact.
#define DENSE_LOAD(SLOT, UR, KR)                                      \
  do {                                                                \
    int ad_[EPT];                                                     \
    bool ok_[EPT], in_[EPT];                                          \
    _Pragma("unroll") for (int q = 0; q < EPT; ++q) {                 \
      const int e = tid + q * NT < TOT ? tid + q * NT : TOT - 1;      \
      int j, c;                                                       \
      DENSE_MAP(e, j, c);                                             \
      const int b = cbase[SLOT][c];                                   \
      ok_[q] = b >= 0 && tid + q * NT < TOT;                          \
      in_[q] = ok_[q] && j != 0 && j != N;                            \
      ad_[q] = ok_[q] ? b + j * stride : 0;                           \
    }                                                                 \
    _Pragma("unroll") for (int q = 0; q < EPT; ++q) {                 \
      UR[q] = a.u[ad_[q]];                                            \
      KR[q] = a.K[ad_[q]];                                            \
    }                                                                 \
    _Pragma("unroll") for (int q = 0; q < EPT; ++q) {                 \
      UR[q] = in_[q] ? UR[q] : T(0);                                  \
      KR[q] = ok_[q] ? KR[q] : T(0);                                  \
    }                                                                 \
  } while (0)

// Persistent: each workgroup walks tiles blockIdx.x, +gridDim.x, ... over the
// interior-transverse pencils and keeps the next tile's u and K loads in flight
// in registers while it computes the current one.  In the first pass it also
// clears the pencils that lie in a face (all their nodes are boundary nodes).
template <typename T, int NC, int MODE, bool FIRST>
__global__ __launch_bounds__(64 * dense_dims(NC).NW) void k_dense_pass(DenseArgs<T> a) {
  constexpr DenseDims S = dense_dims(NC);
  constexpr int N = NC, n = NC + 1;
  constexpr int NT = 64 * S.NW;
  constexpr int C = S.C;
  constexpr int SC = C + 1;  // LDS row stride (odd: conflict-free transposed writes)
  constexpr int TOT = n * C;
  constexpr int EPT = (TOT + NT - 1) / NT;
  constexpr int LPC = pow2_floor(NT / C) < 64 ? pow2_floor(NT / C) : 64;  // lanes per column
  typedef typename Mfma<T>::v4 V4;

  extern __shared__ __align__(16) unsigned char smem[];
  T* tab = (T*)smem;
  T* U = tab + S.TAB;
  T* drw = U + n * SC;  // face rows D[0][:], D[N][:]
  T* cend = drw + 2 * n;
  int(*cbase)[C] = (int(*)[C])(cend + 2 * C);
  const T* amid = tab + S.OFF_MID;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int mt = wave % S.MT, cg = wave / S.MT;
  const int li = lane & 15, lk = lane >> 4;
  const int col = cg * 16 + li;  // this lane's B column / accumulator column
  const int lc = tid / LPC, lg = tid - lc * LPC;
  const int axis = a.axis;
  const int n0 = a.n[0], n1 = a.n[1], n2 = a.n[2];
  const int stride = axis == 2 ? 1 : axis == 1 ? n2 : n1 * n2;
  const bool contig = axis == 2;
  const int nai = (axis == 0 ? n1 : n0) - 2, nbi = (axis == 2 ? n1 : n2) - 2;
  const int npen = nai * nbi;
  const int ntiles = (npen + C - 1) / C;
  const bool nlo = (a.bcmask >> (2 * axis)) & 1, nhi = (a.bcmask >> (2 * axis + 1)) & 1;
  const T* Ao = tab + mt * S.KO4 * 64 + lane;
  const T* Ae = tab + S.OFF_E + mt * S.KE4 * 64 + lane;

  {
    // fragment table and face rows into LDS, loads batched
    constexpr int TI = (S.TAB + NT - 1) / NT;
    T tv[TI];
#pragma unroll
    for (int i = 0; i < TI; ++i) tv[i] = a.tab[tid + i * NT < S.TAB ? tid + i * NT : S.TAB - 1];
    const int jr = tid < n ? tid : n - 1;
    const T r0 = a.drow0[jr], rN = a.drowN[jr];
#pragma unroll
    for (int i = 0; i < TI; ++i)
      if (tid + i * NT < S.TAB) tab[tid + i * NT] = tv[i];
    for (int j = tid; j < n; j += NT) {
      drw[j] = j == jr ? r0 : a.drow0[j];
      drw[n + j] = j == jr ? rN : a.drowN[j];
    }
  }

  if (FIRST) {
    // pencils in a face: every node is a boundary node of the reduced system
    const int na = nai + 2, nb = nbi + 2;
    const int nface = na * nb - npen;
    for (int f = blockIdx.x; f < nface; f += gridDim.x) {
      int ia, ib;
      if (f < 2 * nb) {
        ia = f < nb ? 0 : na - 1;
        ib = f < nb ? f : f - nb;
      } else {
        const int g = f - 2 * nb;
        ia = 1 + (g >> 1);
        ib = (g & 1) ? nb - 1 : 0;
      }
      const int b = axis == 2 ? (ia * n1 + ib) * n2 : axis == 1 ? ia * n1 * n2 + ib : ia * n2 + ib;
      for (int j = tid; j < n; j += NT) a.y[b + j * stride] = T(0);
    }
  }

  int tile = blockIdx.x;
  int slot = 0;
  DENSE_COLS(0, tile);
  __syncthreads();
  T ureg[EPT], kreg[EPT];
  DENSE_LOAD(0, ureg, kreg);

  for (; tile < ntiles; tile += gridDim.x, slot ^= 1) {
    const int nxt = tile + gridDim.x;
    __syncthreads();  // previous tile's readers of U and of slot^1 are done
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = tid + q * NT;
      if (e < TOT) {
        int j, c;
        DENSE_MAP(e, j, c);
        U[j * SC + c] = ureg[q];
      }
    }
    if (nxt < ntiles) DENSE_COLS(slot ^ 1, nxt);
    __syncthreads();

    // in flight during this tile: next tile's u and K (the last tile reloads
    // its own columns), this tile's y
    T unx[EPT], knx[EPT], yreg[EPT];
    DENSE_LOAD(nxt < ntiles ? (slot ^ 1) : slot, unx, knx);
    if (!FIRST) {
      int ad[EPT];
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        const int e = tid + q * NT < TOT ? tid + q * NT : TOT - 1;
        int j, c;
        DENSE_MAP(e, j, c);
        const int b = cbase[slot][c];
        ad[q] = b >= 0 ? b + j * stride : 0;
      }
#pragma unroll
      for (int q = 0; q < EPT; ++q) yreg[q] = a.y[ad[q]];
    }

    if (MODE == DENSE_REDUCED) {
      // homogeneous lift of the end values through the Neumann face rows
      T s0 = T(0), sN = T(0);
      if (lc < C)
        for (int m = 1 + lg; m < N; m += LPC) {
          const T v = U[m * SC + lc];
          s0 += drw[m] * v;
          sN += drw[n + m] * v;
        }
      s0 = group_sum<LPC>(s0);
      sN = group_sum<LPC>(sN);
      if (lc < C && lg == 0) {
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
        U[lc] = u0;
        U[N * SC + lc] = uN;
      }
      __syncthreads();
    }

    V4 acco, acce;
    T midv;
    // first derivative (all n rows)
    DENSE_GEMM(acco, acce);
    DENSE_MID(midv);
    __syncthreads();
    DENSE_EPI(acco, acce, midv);
    __syncthreads();

    // pointwise flux K * (M u)
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = tid + q * NT;
      if (e < TOT) {
        int j, c;
        DENSE_MAP(e, j, c);
        U[j * SC + c] *= kreg[q];
      }
    }
    __syncthreads();

    // divergence part
    DENSE_GEMM(acco, acce);
    DENSE_MID(midv);
    __syncthreads();
    DENSE_EPI(acco, acce, midv);
    __syncthreads();

    if (MODE == DENSE_TRANSPOSE) {
      // transposed lift: mu = M^{-T} [z_0, z_N]; interior -= mu0 D[0][:] + muN D[N][:]
      if (tid < C) {
        const T z0 = U[tid], zN = U[N * SC + tid];
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
        cend[2 * tid] = mu0;
        cend[2 * tid + 1] = muN;
      }
      __syncthreads();
    }

    // store: interior nodes (accumulated), the two end nodes (0); values
    // first, then one unconditional store per element (off-tile ones to the sink)
    {
      T ov[EPT];
      T* op[EPT];
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        const int e = tid + q * NT < TOT ? tid + q * NT : TOT - 1;
        int j, c;
        DENSE_MAP(e, j, c);
        const int b = cbase[slot][c];
        const bool ok = b >= 0 && tid + q * NT < TOT;
        const bool in = j != 0 && j != N;
        T x = U[j * SC + c];
        if (MODE == DENSE_TRANSPOSE) x -= cend[2 * c] * drw[j] + cend[2 * c + 1] * drw[n + j];
        if (!FIRST) x += yreg[q];
        ov[q] = in ? x : T(0);
        op[q] = ok ? a.y + (b + j * stride) : a.sink;
      }
#pragma unroll
      for (int q = 0; q < EPT; ++q) *op[q] = ov[q];
    }
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      ureg[q] = unx[q];
      kreg[q] = knx[q];
    }
  }
}

#undef DENSE_MAP
#undef DENSE_GEMM
#undef DENSE_MID
#undef DENSE_EPI
#undef DENSE_COLS
#undef DENSE_LOAD

}  // namespace cheb
