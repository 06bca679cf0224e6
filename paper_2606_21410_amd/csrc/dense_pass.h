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
// halves the multiply-adds of the dense product.  The tile is kept in LDS in
// split form, e_j in rows j <= N/2 and o_j in rows N/2 + 1 + j, so the matrix
// instructions take their B operands straight from LDS: the loads fetch each
// pencil's nodes j and N - j together, and the first product's epilogue
// writes the flux split the same way.
#pragma once

#include "dev_common.h"
#include "pencil.h"

namespace cheb {

// DENSE_NODE is or-ed into either mode when the plan has per-node Robin
// coefficients: the lift then reads each pencil's own end-block inverse.
// DENSE_DACC (with DENSE_REDUCED, accumulating passes only): y += D (K .* L v)
// on the interior nodes, one derivative of the pointwise product of K with the
// lifted pencil -- the Newton Jacobian's k'(T) term, K standing for
// k'(T) D_a T.  The first product then serves only for the lift's face-row sums.
// DENSE_JAC (with DENSE_REDUCED, 4-wave tiles, FP64): the Newton Jacobian's
// whole axis term, y (+)= D (K .* D L v + C .* L v), the flux epilogue adding
// C .* (lifted v) from a third LDS tile that holds the axis' C = k'(T) D_a T.
enum DenseMode { DENSE_REDUCED = 0, DENSE_TRANSPOSE = 1, DENSE_NODE = 2, DENSE_DACC = 4, DENSE_JAC = 8 };

// element i of a system's field at base (uniform): a system's field stays
// below 4 GiB (at most 129^3 nodes per axis triple), so the byte offset fits
// 32 bits and the address is a scalar base plus one vector offset register
template <typename T>
__device__ __forceinline__ T dense_at(const T* base, int i) {
  return *(const T*)((const char*)base + (unsigned)i * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ T& dense_ref(T* base, unsigned i) {
  return *(T*)((char*)base + i * (unsigned)sizeof(T));
}

// lane move across a DPP pattern (quad permutation, half-row or row mirror)
template <int CTRL>
__device__ __forceinline__ float dpp_move(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// sum over aligned groups of G <= 16 consecutive lanes (within one DPP row),
// left in every lane of the group: swaps within pairs and quads, then the
// half-row mirror pairs the two quads of each 8, the row mirror the two 8s
template <int G, typename T>
__device__ __forceinline__ T row_sum(T v) {
  static_assert(G == 1 || G == 2 || G == 4 || G == 8 || G == 16, "row_sum: group of 1 to 16 lanes");
  if (G >= 2) v += dpp_move<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  if (G >= 4) v += dpp_move<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  if (G >= 8) v += dpp_move<0x141>(v);  // row_half_mirror
  if (G >= 16) v += dpp_move<0x140>(v); // row_mirror
  return v;
}

// Compile-time shape of the split product for one N (also used by the host
// code that writes the fragment tables and sizes the LDS).
struct DenseDims {
  int N, HALF, KO, KE, KO4, KE4, R, RM, MT, WC, NW, C, OFF_E, OFF_MID, OFF_COL, TAB;
  bool EVEN, MIDV;
};

// Two tile shapes: V = 0 keeps the fragment table in LDS and runs 8-wave
// workgroups (one per CU); V = 1 keeps each wave's fragments in registers and
// runs 4-wave workgroups (two per CU, so one overlaps the other's memory phases).
__host__ __device__ constexpr DenseDims dense_dims(int N, int V = 0) {
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
  d.WC = V == 0 ? (d.MT == 3 ? 2 : 8 / d.MT)   // 16-column groups per workgroup
               : (d.MT >= 3 ? 1 : 4 / d.MT);
  d.NW = d.MT * d.WC;                    // waves per workgroup
  d.C = 16 * d.WC;                       // pencils per tile
  // fragment table: [mt][ks][lane] for Ao, then Ae, then the middle row of Ao,
  // then the end columns M[:][0] and M[:][N] (the lift's rank-2 correction)
  d.OFF_E = d.MT * d.KO4 * 64;
  d.OFF_MID = d.OFF_E + d.MT * d.KE4 * 64;
  d.OFF_COL = d.OFF_MID + d.KO4 * 4;
  d.TAB = d.OFF_COL + 2 * (N + 1);
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

// LDS carve of one workgroup (bytes): fragment table, u tile, K tile (and the
// C tile of DENSE_JAC), face rows, the per-column lift values / transposed-lift
// multipliers, column bookkeeping
template <typename T>
__host__ __device__ constexpr int dense_lds_bytes(int N, int V, bool jac = false) {
  const DenseDims d = dense_dims(N, V);
  const int n = N + 1, SC = d.C + 1;
  const int tabl = V == 0 ? d.TAB : d.TAB - d.OFF_MID;  // V = 1: only the middle row and end columns
  return (tabl + (jac ? 3 : 2) * n * SC + 2 * n + 2 * d.C) * (int)sizeof(T) + 2 * d.C * (int)sizeof(int);
}

// one system of a batched pass (same N, box and tile shape as the others): its
// offset in the packed fields, the offset of its conductivity in the packed K
// (systems given the same K, e.g. the load cases of one microstructure, share
// one copy) and its face types
struct DenseSys {
  long long off;
  long long koff;
  int bcmask;
  int pad_;
};

template <typename T>
struct DenseArgs;

// entry i of the active-system list, read through the constant address space
// (scalar loads; the tables are not written while a pass runs)
template <typename T>
__device__ inline DenseSys dense_sys_at(const DenseArgs<T>& a, int i) {
  typedef const __attribute__((address_space(4))) int ci4;
  typedef const __attribute__((address_space(4))) long long cl4;
  const DenseSys* e = a.sys + ((ci4*)a.act)[i];
  DenseSys s;
  s.off = *(cl4*)&e->off;
  s.koff = *(cl4*)&e->koff;
  s.bcmask = *(ci4*)&e->bcmask;
  s.pad_ = 0;
  return s;
}

// one axis of a launch: its tables, the lift's end-block entries and its output
template <typename T>
struct DenseAxis {
  const T* tab;    // fragment table of D (reduced) or D^T (transpose)
  const T* drow0;  // face rows D[0][:], D[N][:] for the lift
  const T* drowN;
  T* y;            // output (single system; batches: the packed base)
  const T* c;      // DENSE_JAC: the axis' coefficient C of the lifted direction; null otherwise
  // per-node Robin coefficients (modes with DENSE_NODE): each pencil's own
  // inverse, 4 entries per pencil of the axis (face numbering), laid out as
  // i00, i0N, iN0, iNN with 1 / m00 or 1 / mNN in place of the inverse when
  // one end is Dirichlet; null otherwise (always for batches)
  const T* rinv;
  // the face rows' 2 x 2 matrix M = [m00 m0N; mN0 mNN] of the lift: the
  // entries of M^{-1} (both ends Neumann) and 1 / m00, 1 / mNN (one end)
  T i00, i0N, iN0, iNN, r00, rNN;
  int axis;
};

template <typename T>
struct DenseArgs {
  const int* gate;  // null, or a device flag: the pass does nothing while it reads 0
  const T* u;  // single system (sys == nullptr)
  const T* K;
  const DenseSys* sys;  // batched: system table (device) and the active systems' indices
  const int* act;
  int nact;
  int n[3];
  int bcmask;  // face types of the single system
  // nseg = 2 (first passes of a single system): the launch serves two axes,
  // ax[0] and ax[1], each into its own output; workgroup b takes axis
  // ax[(b >> 3) & 1], so every XCD holds workgroups of both (the grid is a
  // multiple of 16)
  int nseg;
  // accumulating pass along the unit-stride axis: y += yadd + this pass (yadd
  // is the second output of a two-axis launch); unused by the other passes
  const T* yadd;
  DenseAxis<T> ax[2];
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

// tile pair p -> (row jp <= N/2 of the pair (jp, N - jp), column c), laid
// out like DENSE_MAP
#define DENSE_PMAP(p, jp, c)  \
  do {                        \
    if (contig) {             \
      c = (p) / S.KE;         \
      jp = (p) - c * S.KE;    \
    } else {                  \
      jp = (p) / C;           \
      c = (p) - jp * C;       \
    }                         \
  } while (0)

// ACCO/ACCE = split products of the split LDS tile (B operand: o_j, e_j) with
// this wave's A fragments (from the LDS table).  Rows j > N/2 of the last
// k-step of the even part meet zero table entries.
#define DENSE_GEMM(ACCO, ACCE, ISSUE)                                              \
  do {                                                                             \
    ACCO = V4{0, 0, 0, 0};                                                         \
    ACCE = V4{0, 0, 0, 0};                                                         \
    _Pragma("unroll") for (int ks = 0; ks < S.KE4; ++ks) {                         \
      ISSUE(ks);                                                                   \
      const int j = 4 * ks + lk;                                                   \
      if (ks < S.KO4) ACCO = Mfma<T>::mac(V == 0 ? Ao[ks * 64] : ao[ks], U[(S.KE + j) * SC + col], ACCO); \
      ACCE = Mfma<T>::mac(V == 0 ? Ae[ks * 64] : ae[ks], U[j * SC + col], ACCE);   \
    }                                                                              \
  } while (0)

// vector-ALU dot products of each tile column with the LDS tile for the middle
// row N/2 of the odd part (when it does not fill a 16-row block); every lane of
// each column's group holds the sum.
#define DENSE_VDOT(MIDOUT)                                                         \
  do {                                                                             \
    MIDOUT = T(0);                                                                 \
    if (S.MIDV) {                                                                  \
      if (lc < C)                                                                  \
        for (int j = lg; j < S.KO; j += LPC)                                       \
          MIDOUT += amid[j] * U[(S.KE + j) * SC + lc];                             \
      MIDOUT = row_sum<LPC>(MIDOUT);                                               \
    }                                                                              \
  } while (0)

// face numbering of column c of tile t (the pencil's index among all pencils
// along the axis, which indexes the packed face arrays); 0 past the last pencil
__device__ inline int dense_face_index(int t, int c, int C, int tps, int npen, int nbi) {
  const int q = (t % tps) * C + c;
  return q < npen ? (1 + q / nbi) * (nbi + 2) + 1 + q % nbi : 0;
}

// end values of the homogeneous lift (Section 2.3.1) of each column: the
// first product's rows 0 and N are the face-row dot products s0 = D[0][:] u and
// sN = D[N][:] u of the interior values, and [u0, uN] solves the face rows'
// 2 x 2 system M [u0, uN] = -[s0, sN] on the Neumann ends.  Row 0 sits in
// register r = 0 of the lanes lk == 0 of the waves with mt == 0.
#define DENSE_LIFTVALS(ACCO, ACCE)                                          \
  do {                                                                      \
    if (mt == 0 && lk == 0) {                                               \
      const T s0_ = ACCO[0] + ACCE[0], sN_ = ACCO[0] - ACCE[0];             \
      T u0 = T(0), uN = T(0);                                               \
      if (RN) {                                                             \
        const T* e_ = A.rinv + 4 * dense_face_index(tile, col, C, tps, npen, nbi); \
        u0 = -(e_[0] * s0_ + e_[1] * sN_);                                  \
        uN = -(e_[2] * s0_ + e_[3] * sN_);                                  \
      } else if (nlo && nhi) {                                              \
        u0 = -(A.i00 * s0_ + A.i0N * sN_);                                  \
        uN = -(A.iN0 * s0_ + A.iNN * sN_);                                  \
      } else if (nlo) {                                                     \
        u0 = -A.r00 * s0_;                                                  \
      } else if (nhi) {                                                     \
        uN = -A.rNN * sN_;                                                  \
      }                                                                     \
      cend[2 * col] = u0;                                                   \
      cend[2 * col + 1] = uN;                                               \
    }                                                                       \
  } while (0)

// accumulators -> LDS tile rows i and N-i.  FLUX (first product): add the
// lift's rank-2 correction u0 M[:][0] + uN M[:][N] (LIFT, on axes with a
// Neumann end), multiply by K and store the flux split into the u tile.  With
// DACC the first product's rows are not used: rows i and N-i are the lifted
// pencil itself, (e_i +- o_i) / 2 from the split tile (u0 and uN at i = 0),
// times K.  M is
// centro-antisymmetric, so row N-i of the correction is -(u0 M[i][N] +
// uN M[i][0]).  Otherwise (second product) the rows go to the K tile, dead
// since the first epilogue, so the second product's reads of the u tile need
// no barrier before this.
#define DENSE_EPI(ACCO, ACCE, MIDVAL, FLUX, LIFT)                            \
  do {                                                                       \
    T u0_ = T(0), uN_ = T(0);                                                \
    const bool lift_ = (LIFT) && (nlo || nhi);                               \
    if (lift_) {                                                             \
      u0_ = cend[2 * col];                                                   \
      uN_ = cend[2 * col + 1];                                               \
    }                                                                        \
    _Pragma("unroll") for (int r = 0; r < 4; ++r) {                          \
      const int i = 16 * mt + Mfma<T>::row(lk, r);                           \
      if (i < S.RM) {                                                        \
        const T o = ACCO[r], e = ACCE[r];                                    \
        T lo = o + e, hi = o - e;                                            \
        if (DACC && (FLUX)) {                                                \
          if (i == 0) {                                                      \
            lo = cend[2 * col];                                              \
            hi = cend[2 * col + 1];                                          \
          } else {                                                           \
            const T ev_ = U[i * SC + col];                                   \
            const T od_ = 2 * i == N ? T(0) : U[(S.KE + i) * SC + col];      \
            lo = T(0.5) * (ev_ + od_);                                       \
            hi = T(0.5) * (ev_ - od_);                                       \
          }                                                                  \
        } else if (lift_) {                                                  \
          const T c0_ = dc0[i], cN_ = dcN[i];                                \
          lo += u0_ * c0_ + uN_ * cN_;                                       \
          hi -= u0_ * cN_ + uN_ * c0_;                                       \
        }                                                                    \
        if (FLUX) {                                                          \
          /* flux K * (M u), stored split for the second product */          \
          T vlo_ = T(0), vhi_ = T(0);                                        \
          if (JAC) {                                                         \
            /* the lifted pencil itself, before its rows are overwritten */  \
            if (i == 0) {                                                    \
              vlo_ = cend[2 * col];                                          \
              vhi_ = cend[2 * col + 1];                                      \
            } else {                                                         \
              const T ev_ = U[i * SC + col];                                 \
              const T od_ = 2 * i == N ? T(0) : U[(S.KE + i) * SC + col];    \
              vlo_ = T(0.5) * (ev_ + od_);                                   \
              vhi_ = T(0.5) * (ev_ - od_);                                   \
            }                                                                \
          }                                                                  \
          lo *= Kt[i * SC + col];                                            \
          hi *= Kt[(N - i) * SC + col];                                      \
          if (JAC) {                                                         \
            lo += Ct[i * SC + col] * vlo_;                                   \
            hi += Ct[(N - i) * SC + col] * vhi_;                             \
          }                                                                  \
          if (2 * i == N) {                                                  \
            U[i * SC + col] = lo + lo;                                       \
          } else {                                                           \
            U[i * SC + col] = lo + hi;                                       \
            U[(S.KE + i) * SC + col] = lo - hi;                              \
          }                                                                  \
        } else if (2 * i == N) {                                             \
          Kt[i * SC + col] = lo;                                             \
        } else {                                                             \
          Kt[i * SC + col] = lo;                                             \
          Kt[(N - i) * SC + col] = hi;                                       \
        }                                                                    \
      }                                                                      \
    }                                                                        \
    if (S.MIDV && lc < C && lg == 0) {                                       \
      T m_ = MIDVAL;                                                         \
      if (DACC && (FLUX)) m_ = T(0.5) * U[S.HALF * SC + lc];                 \
      else if (lift_) m_ += cend[2 * lc] * dc0[S.HALF] + cend[2 * lc + 1] * dcN[S.HALF]; \
      if (FLUX) m_ *= Kt[S.HALF * SC + lc];                                  \
      if (JAC && (FLUX)) m_ += Ct[S.HALF * SC + lc] * (T(0.5) * U[S.HALF * SC + lc]); \
      if (FLUX) U[S.HALF * SC + lc] = m_ + m_;                               \
      else Kt[S.HALF * SC + lc] = m_;                                        \
    }                                                                        \
  } while (0)

// column bookkeeping of tile TILE into slot SLOT: linear offset of each
// interior-transverse pencil's first node, -1 past the last pencil
#define DENSE_COLS(SLOT, TILE)                                             \
  do {                                                                     \
    if (tid < C) {                                                         \
      const int q_ = ((TILE) % tps) * C + tid;                             \
      int b_ = -1;                                                         \
      if (q_ < npen) {                                                     \
        const int ia_ = 1 + q_ / nbi, ib_ = 1 + (q_ - (q_ / nbi) * nbi);   \
        b_ = axis == 2 ? (ia_ * n1 + ib_) * n2 : axis == 1 ? ia_ * n1 * n2 + ib_ : ia_ * n2 + ib_; \
      }                                                                    \
      cbase[SLOT][tid] = b_;                                               \
    }                                                                      \
  } while (0)

// global -> registers: u and K of the tile in slot SLOT, pair by pair (nodes
// jp and N - jp of a pencil; u's end nodes are cleared when the tile is written
// to LDS).  Every load is issued (off-tile pairs read node 0 and their columns
// are discarded), so the number of outstanding loads is static and the
// compiler's waits stay exact; nothing here waits for the loads.
#define DENSE_LOAD(SLOT, UR, KR, PU, PK, CR, PC)                      \
  do {                                                                \
    int alo_[EPP], ahi_[EPP];                                         \
    _Pragma("unroll") for (int q = 0; q < EPP; ++q) {                 \
      const int p = tid + q * NT < TOTP ? tid + q * NT : TOTP - 1;    \
      int jp, c;                                                      \
      DENSE_PMAP(p, jp, c);                                           \
      const int b = cbase[SLOT][c];                                   \
      alo_[q] = b >= 0 ? b + jp * stride : 0;                         \
      ahi_[q] = b >= 0 ? b + (N - jp) * stride : 0;                   \
    }                                                                 \
    _Pragma("unroll") for (int q = 0; q < EPP; ++q) {                 \
      UR[2 * q] = dense_at(PU, alo_[q]);                              \
      UR[2 * q + 1] = dense_at(PU, ahi_[q]);                          \
      KR[2 * q] = dense_at(PK, alo_[q]);                              \
      KR[2 * q + 1] = dense_at(PK, ahi_[q]);                          \
      if (JAC) {                                                      \
        CR[JAC ? 2 * q : 0] = dense_at(PC, alo_[q]);                  \
        CR[JAC ? 2 * q + 1 : 0] = dense_at(PC, ahi_[q]);              \
      }                                                               \
    }                                                                 \
  } while (0)

// pointers and face types of the system that owns tile TILE (uniform, so the
// tables are read with scalar loads, which wait on nothing in the vector queue)
#define DENSE_SYS(TILE, PU, PK, PY, BM)                   \
  do {                                                    \
    if (a.sys) {                                          \
      const DenseSys s_ = dense_sys_at(a, (TILE) / tps);  \
      PU = a.u + s_.off;                                  \
      PK = a.K + s_.koff;                                 \
      PY = A.y + s_.off;                                  \
      BM = s_.bcmask;                                     \
    } else {                                              \
      PU = a.u;                                           \
      PK = a.K;                                           \
      PY = A.y;                                           \
      BM = a.bcmask;                                      \
    }                                                     \
  } while (0)

// Persistent: each workgroup walks its XCD's contiguous range of tiles over
// the interior-transverse pencils (in a two-axis launch, within its axis'
// half of the grid) and, with V = 0, keeps the next tile's u and K loads in
// flight in registers while it computes the current one.  A first pass also
// clears the pencils of its axis that lie in a face (all their nodes are
// boundary nodes).  The accumulating pass along the unit-stride axis adds the
// second partial sum yadd of a two-axis launch.
template <typename T, int NC, int MODE, bool FIRST, int V, bool CG>
__global__ __launch_bounds__(64 * dense_dims(NC, V).NW, 2) void k_dense_pass(DenseArgs<T> a) {
  if (a.gate && !*a.gate) return;
  constexpr int BASE = MODE & 1;                   // DENSE_REDUCED or DENSE_TRANSPOSE
  constexpr bool RN = (MODE & DENSE_NODE) != 0;    // per-pencil end-block inverses
  constexpr bool DACC = (MODE & DENSE_DACC) != 0;  // one derivative of K .* (lifted u)
  constexpr bool JAC = (MODE & DENSE_JAC) != 0;    // reduced operator plus C .* (lifted u) in the flux
  static_assert(!JAC || (BASE == DENSE_REDUCED && !DACC && V == 1), "DENSE_JAC: reduced passes, 4-wave tiles");
  static_assert(!DACC || (BASE == DENSE_REDUCED && !FIRST), "DENSE_DACC: accumulating reduced passes only");
  constexpr bool YADD = CG && !FIRST && !DACC;     // the last pass of a two-axis apply adds yadd
  constexpr DenseDims S = dense_dims(NC, V);
  constexpr int N = NC, n = NC + 1;
  constexpr int NT = 64 * S.NW;
  constexpr int C = S.C;
  constexpr int SC = C + 1;  // LDS row stride (odd: conflict-free transposed writes)
  constexpr int TOT = n * C;
  constexpr int EPT = (TOT + NT - 1) / NT;
  static_assert(N % 2 == 0, "split tile layout needs even N");
  constexpr int TOTP = S.KE * C;                 // node pairs (jp, N - jp) of a tile
  constexpr int EPP = (TOTP + NT - 1) / NT;      // pairs per thread
  constexpr int NL = 4 * EPP;                    // u and K loads per thread
  constexpr int LPC = pow2_floor(NT / C) < 64 ? pow2_floor(NT / C) : 64;  // lanes per column
  typedef typename Mfma<T>::v4 V4;

  extern __shared__ __align__(16) unsigned char smem[];
  // V = 0: whole table in LDS; V = 1: LDS holds the table from OFF_MID on
  constexpr int TB = V == 0 ? 0 : S.OFF_MID;  // first table entry kept in LDS
  T* tab = (T*)smem - TB;
  T* U = tab + S.TAB;
  T* Kt = U + n * SC;
  T* Ct = Kt + n * SC;   // DENSE_JAC: the C tile (natural node order, like K)
  T* drw = Ct + (JAC ? n * SC : 0);  // face rows D[0][:], D[N][:]
  T* cend = drw + 2 * n;
  int(*cbase)[C] = (int(*)[C])(cend + 2 * C);
  const T* amid = tab + S.OFF_MID;
  const T* dc0 = tab + S.OFF_COL;  // end columns M[:][0], M[:][N]
  const T* dcN = dc0 + n;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int mt = wave % S.MT, cg = wave / S.MT;
  const int li = lane & 15, lk = lane >> 4;
  const int col = cg * 16 + li;  // this lane's B column / accumulator column
  const int lc = tid / LPC, lg = tid - lc * LPC;
  // segment of a two-axis launch, and this workgroup's index and the grid size
  // within it (XCD bits kept: vb & 7 == blockIdx.x & 7)
  const int seg = a.nseg == 2 ? (blockIdx.x >> 3) & 1 : 0;
  const int vb = a.nseg == 2 ? (int)(((blockIdx.x >> 4) << 3) | (blockIdx.x & 7)) : (int)blockIdx.x;
  const int vg = a.nseg == 2 ? (int)(gridDim.x >> 1) : (int)gridDim.x;
  const DenseAxis<T> A = seg ? a.ax[1] : a.ax[0];
  const int axis = A.axis;
  const int n0 = a.n[0], n1 = a.n[1], n2 = a.n[2];
  // CG: the pass runs along the unit-stride axis (axis 2)
  const int stride = CG ? 1 : axis == 1 ? n2 : n1 * n2;
  constexpr bool contig = CG;
  const int nai = (axis == 0 ? n1 : n0) - 2, nbi = (axis == 2 ? n1 : n2) - 2;
  const int npen = nai * nbi;
  const int tps = (npen + C - 1) / C;  // tiles per system
  const int nsys = a.sys ? a.nact : 1;
  const int ntiles = nsys * tps;
  bool nlo = false, nhi = false;
  const T* Ao = tab + mt * S.KO4 * 64 + lane;
  const T* Ae = tab + S.OFF_E + mt * S.KE4 * 64 + lane;
  T ao[V == 1 ? S.KO4 : 1], ae[V == 1 ? S.KE4 : 1];
  if (V == 1) {
#pragma unroll
    for (int ks = 0; ks < S.KO4; ++ks) ao[ks] = A.tab[(mt * S.KO4 + ks) * 64 + lane];
#pragma unroll
    for (int ks = 0; ks < S.KE4; ++ks) ae[ks] = A.tab[S.OFF_E + (mt * S.KE4 + ks) * 64 + lane];
  }

  if (FIRST) {
    // pencils in a face: every node is a boundary node of the reduced system
    const int na = nai + 2, nb = nbi + 2;
    const int nface = na * nb - npen;
    for (int fs = vb; fs < nsys * nface; fs += vg) {
      const int f = fs % nface;
      T* ys = a.sys ? A.y + a.sys[a.act[fs / nface]].off : A.y;
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
      for (int j = tid; j < n; j += NT) ys[b + j * stride] = T(0);
    }
  }

  // prologue: fragment-table loads, then the first tile's loads, both in
  // flight before the table is written to LDS
  constexpr int TI = (S.TAB - TB + NT - 1) / NT;
  T tv[TI];
#pragma unroll
  for (int i = 0; i < TI; ++i) tv[i] = A.tab[TB + (tid + i * NT < S.TAB - TB ? tid + i * NT : S.TAB - TB - 1)];
  const int jr = tid < n ? tid : n - 1;
  const T r0v = A.drow0[jr], rNv = A.drowN[jr];
  // XCD-aware tile order: workgroups are dealt round-robin to the 8 XCDs, so
  // workgroup b serves a contiguous range of tiles of XCD b % 8 and tiles that
  // share cache lines at their edges meet in the same L2
  int t_step = vg, t_end = ntiles, tile = vb;
  if ((vg & 7) == 0 && ntiles >= vg) {
    const int per = (ntiles + 7) >> 3;
    const int x = vb & 7;
    tile = x * per + (vb >> 3);
    t_step = vg >> 3;
    t_end = min(ntiles, (x + 1) * per);
  }
  int slot = 0;
  DENSE_COLS(0, tile);
  const T *cu, *cK, *nu, *nK;
  T* cy;
  int cbm;
  DENSE_SYS(tile < ntiles ? tile : 0, cu, cK, cy, cbm);
  nu = cu;
  nK = cK;
  lds_barrier();
  // V = 0 loads the next tile's u and K into registers between the first
  // product's matrix instructions and writes them to LDS at the top of the next
  // tile.  V = 1, whose registers hold the fragments, loads each tile at its
  // top and relies on the second workgroup of the CU for overlap: prefetching
  // into registers (during the first product, or after the second epilogue)
  // and into a second LDS buffer pair all measured slower at 129^3.
  constexpr bool PREF = V == 0;
  T ureg[2 * EPP], kreg[2 * EPP], creg[JAC ? 2 * EPP : 1];
  if (PREF) DENSE_LOAD(0, ureg, kreg, cu, cK, creg, A.c);
#pragma unroll
  for (int i = 0; i < TI; ++i)
    if (tid + i * NT < S.TAB - TB) tab[TB + tid + i * NT] = tv[i];
  if (tid < n) {
    drw[tid] = r0v;
    drw[n + tid] = rNv;
  }
  for (int j = tid + NT; j < n; j += NT) {
    drw[j] = A.drow0[j];
    drw[n + j] = A.drowN[j];
  }
  // registers -> LDS: u in split form (e_jp in row jp, o_jp in row N/2 + 1 + jp)
  // with its end nodes cleared (the interior values of the lift), K as it is.
  // Every pair is written, past the tile's last pair to the padding column C,
  // which nothing reads: under a branch the compiler would sink the tail's
  // loads into it and wait for them in a second round trip.
#define DENSE_PUT(DU, UR, KR)                                 \
  do {                                                        \
    _Pragma("unroll") for (int q = 0; q < EPP; ++q) {         \
      const int p = tid + q * NT;                             \
      int jp = 0, c = C;                                      \
      if (p < TOTP) DENSE_PMAP(p, jp, c);                     \
      const T ua = jp != 0 ? UR[2 * q] : T(0);                \
      const T ub = jp != 0 ? UR[2 * q + 1] : T(0);            \
      (DU)[jp * SC + c] = ua + ub;                            \
      if (2 * jp != N) (DU)[(S.KE + jp) * SC + c] = ua - ub;  \
      Kt[jp * SC + c] = KR[2 * q];                            \
      Kt[(N - jp) * SC + c] = KR[2 * q + 1];                  \
      if (JAC) {                                              \
        Ct[jp * SC + c] = creg[JAC ? 2 * q : 0];              \
        Ct[(N - jp) * SC + c] = creg[JAC ? 2 * q + 1 : 0];    \
      }                                                       \
    }                                                         \
  } while (0)

  for (; tile < t_end; tile += t_step, slot ^= 1) {
    const int nxt = tile + t_step < t_end ? tile + t_step : ntiles;
    lds_barrier();  // previous tile's readers of U and of slot^1 are done
    DENSE_SYS(tile, cu, cK, cy, cbm);
    nlo = (cbm >> (2 * axis)) & 1;
    nhi = (cbm >> (2 * axis + 1)) & 1;
    if (!PREF) DENSE_LOAD(slot, ureg, kreg, cu, cK, creg, A.c);
    DENSE_PUT(U, ureg, kreg);
    if (nxt < ntiles) DENSE_COLS(slot ^ 1, nxt);
    else if (tid < C) cbase[slot ^ 1][tid] = -1;  // loads of the next tile all read node 0
    lds_barrier();

    // in flight during this tile: next tile's u and K (V = 0), this tile's y.  Their
    // addresses are formed here and the loads are issued a few at a time
    // between the products' matrix instructions, so the matrix cores keep
    // working while load issue waits for queue space.
    T unx[PREF ? 2 * EPP : 1], knx[PREF ? 2 * EPP : 1], yreg[EPT], y2reg[YADD ? EPT : 1];
    {
      T* ny_;
      int nbm_;
      DENSE_SYS(nxt < ntiles ? nxt : tile, nu, nK, ny_, nbm_);
      (void)ny_;
      (void)nbm_;
    }
    // global offset of element q of the tile in slot SL (node 0 off the tile)
#define DENSE_AD(SL, q)                                                      \
  ([&]() {                                                                   \
    const int e_ = tid + (q) * NT < TOT ? tid + (q) * NT : TOT - 1;          \
    int j_, c_;                                                              \
    DENSE_MAP(e_, j_, c_);                                                   \
    const int b_ = cbase[SL][c_];                                            \
    return b_ >= 0 ? b_ + j_ * stride : 0;                                   \
  }())
    // global offset of node jp (HI: N - jp) of pair q of the tile in slot SL
#define DENSE_PAD(SL, q, HI)                                                 \
  ([&]() {                                                                   \
    const int p_ = tid + (q) * NT < TOTP ? tid + (q) * NT : TOTP - 1;        \
    int jp_, c_;                                                             \
    DENSE_PMAP(p_, jp_, c_);                                                 \
    const int b_ = cbase[SL][c_];                                            \
    return b_ >= 0 ? b_ + ((HI) ? N - jp_ : jp_) * stride : 0;               \
  }())
    // prefetch load L of the next tile: pair L / 4, u_jp, u_{N-jp}, K_jp, K_{N-jp}
#define DENSE_PREF1(L)                                                                     \
  do {                                                                                     \
    const int q_ = PREF ? (L) / 4 : 0;                                                     \
    if ((L) % 4 == 0) unx[PREF ? 2 * q_ : 0] = nu[DENSE_PAD(slot ^ 1, q_, false)];         \
    else if ((L) % 4 == 1) unx[PREF ? 2 * q_ + 1 : 0] = nu[DENSE_PAD(slot ^ 1, q_, true)]; \
    else if ((L) % 4 == 2) knx[PREF ? 2 * q_ : 0] = nK[DENSE_PAD(slot ^ 1, q_, false)];    \
    else knx[PREF ? 2 * q_ + 1 : 0] = nK[DENSE_PAD(slot ^ 1, q_, true)];                   \
  } while (0)
    // loads issued at k-step KS of the first product: prefetch load KS; y loads
    // go between the second product's k-steps
#define DENSE_ISSUE1(KS)                     \
  do {                                       \
    if (PREF && (KS) < NL) DENSE_PREF1(KS);  \
  } while (0)
#define DENSE_ISSUE2(KS)                                              \
  do {                                                                \
    if (!FIRST && (KS) < EPT) {                                       \
      const int q_ = (KS) < EPT ? (KS) : 0;                           \
      const int o_ = DENSE_AD(slot, q_);                              \
      yreg[q_] = dense_at(cy, o_);                                    \
      if (YADD) y2reg[YADD ? q_ : 0] = dense_at(a.yadd, o_);          \
    }                                                                 \
  } while (0)

    V4 acco, acce;
    T midv;
    // first derivative of the lifted pencil (all n rows), then the flux K * (M u)
    DENSE_GEMM(acco, acce, DENSE_ISSUE1);
    // whatever did not fit between the k-steps
#pragma unroll
    for (int ks = S.KE4; ks < (PREF ? NL : 0); ++ks) DENSE_PREF1(ks);
    if (DACC) midv = T(0);  // the middle row comes from the tile itself
    else DENSE_VDOT(midv);
    if (BASE == DENSE_REDUCED) DENSE_LIFTVALS(acco, acce);
    lds_barrier();
    DENSE_EPI(acco, acce, midv, true, BASE == DENSE_REDUCED);
    lds_barrier();

    // divergence part
    DENSE_GEMM(acco, acce, DENSE_ISSUE2);
#pragma unroll
    for (int q = S.KE4; q < EPT; ++q)
      if (!FIRST) {
        const int o_ = DENSE_AD(slot, q);
        yreg[q] = dense_at(cy, o_);
        if (YADD) y2reg[YADD ? q : 0] = dense_at(a.yadd, o_);
      }
    DENSE_VDOT(midv);
    DENSE_EPI(acco, acce, midv, false, false);  // into the K tile: no barrier needed before it
    lds_barrier();

    if (BASE == DENSE_TRANSPOSE) {
      // transposed lift: mu = M^{-T} [z_0, z_N]; interior -= mu0 D[0][:] + muN D[N][:]
      if (tid < C) {
        const T z0 = Kt[tid], zN = Kt[N * SC + tid];
        T mu0 = T(0), muN = T(0);
        if (RN) {
          const T* e = A.rinv + 4 * dense_face_index(tile, tid, C, tps, npen, nbi);
          mu0 = e[0] * z0 + e[2] * zN;
          muN = e[1] * z0 + e[3] * zN;
        } else if (nlo && nhi) {
          mu0 = A.i00 * z0 + A.iN0 * zN;
          muN = A.i0N * z0 + A.iNN * zN;
        } else if (nlo) {
          mu0 = A.r00 * z0;
        } else if (nhi) {
          muN = A.rNN * zN;
        }
        cend[2 * tid] = mu0;
        cend[2 * tid + 1] = muN;
      }
      lds_barrier();
    }

    // store: interior nodes (accumulated), the two end nodes (0); values
    // first, then one unconditional store per element.  Off-tile elements
    // store 0 to the system's node 0, a corner, whose value in the reduced
    // operator's output is 0.
    {
      T ov[EPT];
      unsigned op[EPT];
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        const int e = tid + q * NT < TOT ? tid + q * NT : TOT - 1;
        int j, c;
        DENSE_MAP(e, j, c);
        const int b = cbase[slot][c];
        const bool ok = b >= 0 && tid + q * NT < TOT;
        const bool in = j != 0 && j != N;
        T x = Kt[j * SC + c];
        if (BASE == DENSE_TRANSPOSE && (nlo || nhi)) x -= cend[2 * c] * drw[j] + cend[2 * c + 1] * drw[n + j];
        if (!FIRST) x += yreg[q];
        if (YADD) x += y2reg[YADD ? q : 0];
        ov[q] = in ? x : T(0);
        op[q] = ok ? (unsigned)(b + j * stride) : 0u;
        if (!ok) ov[q] = T(0);
      }
#pragma unroll
      for (int q = 0; q < EPT; ++q) dense_ref(cy, op[q]) = ov[q];
    }
    if (PREF) {
#pragma unroll
      for (int q = 0; q < 2 * EPP; ++q) {
        ureg[q] = unx[PREF ? q : 0];
        kreg[q] = knx[PREF ? q : 0];
      }
    }
  }
}

#undef DENSE_MAP
#undef DENSE_GEMM
#undef DENSE_ISSUE1
#undef DENSE_PREF1
#undef DENSE_PAD
#undef DENSE_PMAP
#undef DENSE_PUT
#undef DENSE_AD
#undef DENSE_ISSUE2
#undef DENSE_VDOT
#undef DENSE_LIFTVALS
#undef DENSE_EPI
#undef DENSE_COLS
#undef DENSE_LOAD
#undef DENSE_SYS

}  // namespace cheb
