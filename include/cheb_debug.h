/*
 * cheb_debug.h - diagnostic entry points of libchebfft.so (not part of the
 * solver's interface): the stream-copy kernel that the attainable HBM
 * bandwidth is measured with, and the matrix-core GEMM of the preconditioner
 * exposed for its lane-layout test.  Conventions as in cheb.h.
 */
#ifndef CHEB_DEBUG_H_
#define CHEB_DEBUG_H_

#include "cheb.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Copy of n doubles, src -> dst (device arrays, 16-byte aligned, not
 * overlapping), by the library's stream-copy kernel: 16-byte loads and stores
 * in a grid-stride loop.  The attainable HBM bandwidth the operator's roofline
 * fraction is also quoted against (2 n * 8 bytes moved).  Asynchronous on
 * `stream`. */
int cheb_debug_copy(const void* src, void* dst, size_t n, void* stream);

/* Dense GEMM on the matrix cores, D (I x C) = A (I x K) B (K x C), row-major
 * device arrays (double for CHEB_F64, float for CHEB_F32).  This is the
 * contraction kernel of the preconditioner, exposed so its MFMA lane layout can
 * be checked directly.  Asynchronous on `stream`. */
int cheb_debug_gemm(int32_t precision, const void* A, const void* B, void* D, int32_t I, int32_t K, int32_t C,
                    void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CHEB_DEBUG_H_ */
