// Pencil bookkeeping shared by the axis-pass and lift kernels: which global
// pencil a tile slot holds, where it starts in memory, and which equations its
// nodes carry.
#pragma once

#include <hip/hip_runtime.h>

namespace cheb {

enum PencilFlag { PF_VALID = 1, PF_TIN = 2, PF_OWN_LO = 4, PF_OWN_HI = 8 };

// Pencils along `axis` are numbered by their two transverse indices (lower
// axis slower).  Returns the flags and the linear offset of the pencil's first
// node.  PF_TIN: both transverse indices interior (its inner nodes are
// interior nodes).  PF_OWN_LO/HI: the end node's equation belongs to this
// axis' face: a node on several faces is owned by the Dirichlet face of lowest
// axis if any, else by the Neumann face of lowest axis.
__host__ __device__ inline int sel3(int a0, int a1, int a2, int i) { return i == 0 ? a0 : i == 1 ? a1 : a2; }

// bcmask: bit f set when face f is Neumann
__host__ __device__ inline int pencil_flags(int axis, int p, int npencils, int n0, int n1, int n2, int bcmask,
                                            long long* base) {
  *base = 0;
  if (p >= npencils) return 0;
  int fl = PF_VALID;
  int ta, tb, ia, ib;
  if (axis == 2) {
    ta = 0; tb = 1; ia = p / n1; ib = p - ia * n1;
    *base = (long long)p * n2;
  } else if (axis == 1) {
    ta = 0; tb = 2; ia = p / n2; ib = p - ia * n2;
    *base = (long long)ia * n1 * n2 + ib;
  } else {
    ta = 1; tb = 2; ia = p / n2; ib = p - ia * n2;
    *base = (long long)p;
  }
  bool hasD = false, hasDlow = false, haslow = false, any = false;
  for (int s = 0; s < 2; ++s) {
    const int bax = s == 0 ? ta : tb, idx = s == 0 ? ia : ib;
    int f = -1;
    if (idx == 0) f = 2 * bax;
    else if (idx == sel3(n0, n1, n2, bax) - 1) f = 2 * bax + 1;
    if (f >= 0) {
      any = true;
      const bool d = ((bcmask >> f) & 1) == 0;
      hasD = hasD || d;
      if (bax < axis) {
        haslow = true;
        hasDlow = hasDlow || d;
      }
    }
  }
  if (!any) fl |= PF_TIN;
  const bool dlo = ((bcmask >> (2 * axis)) & 1) == 0, dhi = ((bcmask >> (2 * axis + 1)) & 1) == 0;
  if (dlo ? !hasDlow : (!hasD && !haslow)) fl |= PF_OWN_LO;
  if (dhi ? !hasDlow : (!hasD && !haslow)) fl |= PF_OWN_HI;
  return fl;
}

__host__ __device__ inline int bc_mask(const int* bc) {
  int m = 0;
  for (int f = 0; f < 6; ++f)
    if (bc[f] == 1) m |= 1 << f;
  return m;
}

__host__ __device__ inline long long pencil_stride(int axis, const int* n) {
  return axis == 2 ? 1LL : axis == 1 ? (long long)n[2] : (long long)n[1] * n[2];
}

__host__ __device__ inline int pencil_count(int axis, const int* n) {
  return axis == 2 ? n[0] * n[1] : axis == 1 ? n[0] * n[2] : n[1] * n[2];
}

// offset of face f's block in the packed face layout (faces x_lo .. z_hi, each
// indexed like the pencils along its axis)
__host__ __device__ inline long long face_offset(int f, const int* n) {
  long long off = 0;
  for (int q = 0; q < f; ++q) off += pencil_count(q / 2, n);
  return off;
}

}  // namespace cheb
