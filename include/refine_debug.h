/*
 * refine_debug.h -- diagnostic entry point of librefine.so for tests.
 *
 * Not an operation of the method and not part of the refinement interface
 * of refine.h: it only lets a test read intermediate quantities of the last
 * step (the product W = A X of Algorithm 4's first line, its low part in the
 * split form, the k x k work area) to compare them with an independent
 * computation.  Nothing in the library depends on it.
 */
#ifndef REFINE_DEBUG_H
#define REFINE_DEBUG_H

#include <stdint.h>

#include "refine.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Writes up to `count` DEVICE addresses of the workspace of a single-problem
 * context to out[0..count-1], in this order: W (n x k row-major, ld k), W_lo
 * (split form only, else NULL), the unnormalised update (n x k), the k x k
 * area (14 k x k blocks), the per-column vectors (6 x k), the control word,
 * the K-split partials of W (NULL without a K split), the row-block partials
 * and the Gram partials.  The addresses stay owned by the context and valid
 * until refine_destroy; read them after synchronising its stream.  Returns
 * REFINE_OK, or REFINE_EINVAL for a NULL context or out, or count < 1. */
int refine_debug_workspace(const refine_ctx* ctx, void** out, int32_t count);

#ifdef __cplusplus
}
#endif

#endif /* REFINE_DEBUG_H */
