/* gtscript_abi.h -- C ABI of the stencil libraries the GTScript-like
 * frontend generates (paper_2311_08322_amd/frontend).
 *
 * The GT4Py paper (Sec. 2.3) describes a toolchain in which a frontend turns
 * a Python stencil definition into an internal representation, an analysis
 * pipeline lowers it, and a backend generates, compiles and loads the
 * implementation, cached under a fingerprint of the definition.  Here the
 * backend writes HIP for gfx950, compiles it with hipcc into one shared
 * library per (definition, dtype) and loads it; every such library exports
 * the functions below with plain C types (no torch types).
 *
 * Fields are passed in the stencil's signature order, scalars likewise (as
 * double; a binary32 library rounds each once).  All device memory belongs to
 * the caller; the library allocates nothing and keeps no state besides the
 * thread-local error text.  Calls are asynchronous on `stream`.
 */
#ifndef GTSCRIPT_ABI_H
#define GTSCRIPT_ABI_H

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  void* data;        /* device pointer of the element at compute-domain point (0,0,0) */
  int64_t stride[3]; /* in elements, order (i, j, k); stride[0] must be 1 */
  int64_t lo[3];     /* points the field holds below the domain origin per axis (>= 0) */
  int64_t hi[3];     /* points from the origin on: indices [-lo, hi) are valid */
} gts_field;

/* Status codes (0 = success). */
#define GTS_OK 0
#define GTS_E_NULL -1      /* a NULL pointer where a field, domain or workspace is needed */
#define GTS_E_ARG -2       /* wrong number of fields or scalars, or a negative extent */
#define GTS_E_STRIDE -3    /* stride[0] != 1 or strides that make rows or levels overlap */
#define GTS_E_HALO -4      /* a field does not cover the points the stencil reads or writes */
#define GTS_E_WORKSPACE -5 /* workspace smaller than gts_workspace_bytes(domain) */
#define GTS_E_LEVELS -6    /* a vertical access leaves its range for this nk (temporary
                              levels, or a sweep reading a level it has not computed) */
#define GTS_E_HIP -7       /* a HIP launch error */

/* Runs the stencil on `domain` (ni, nj, nk).  Fields: nfields descriptors in
 * signature order, each covering the offsets the stencil reads (and the
 * domain where it writes); scalars: nscalars values.  workspace: device
 * memory of gts_workspace_bytes(domain) bytes for temporaries that cross
 * computations (NULL when that is 0), 256-byte aligned.  Output fields may
 * not overlap inputs (not checked: the caller owns aliasing). */
int gts_run(const gts_field* fields, int nfields, const double* scalars, int nscalars,
            const int64_t domain[3], void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Workspace bytes for a domain (0 if the stencil keeps every temporary on chip). */
size_t gts_workspace_bytes(const int64_t domain[3]);

/* "name|fields,...|scalars,...|dtype|fingerprint" of the definition compiled in. */
const char* gts_signature(void);

/* Text of the last error on this thread ("" if none). */
const char* gts_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GTSCRIPT_ABI_H */
