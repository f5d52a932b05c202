/*
 * stencil.h -- C ABI of the MI355X (gfx950) stencil library (libgt4mi.so).
 *
 * What is computed: the two benchmark stencils the GT4Py paper names in
 * Sec. 3.1, a multi-stage horizontal diffusion and an implicit vertical
 * advection.  The paper prints no formulas; these are the benchmark
 * workload's definitions of the two stencils, taken literally:
 *
 *   horizontal diffusion (hdiff), per level k, over the interior I:
 *     lap(i,j) = 4u(i,j) - u(i-1,j) - u(i+1,j) - u(i,j-1) - u(i,j+1)
 *     fx(i,j)  = lap(i+1,j) - lap(i,j), set to 0 where fx*(u(i+1,j)-u(i,j)) > 0
 *     fy(i,j)  = lap(i,j+1) - lap(i,j), set to 0 where fy*(u(i,j+1)-u(i,j)) > 0
 *     out(i,j) = u(i,j) - coeff*(fx(i,j) - fx(i-1,j) + fy(i,j) - fy(i,j-1))
 *   vertical advection (vadv), per column, r = dt_dz:
 *     a_k = -r/4 w_k (k >= 1), a_0 = 0;  c_k = r/4 w_{k+1} (k <= nk-2),
 *     c_{nk-1} = 0;  b_k = 1 + |a_k| + |c_k|;  d_k = u_k + data_k;
 *     solve a_k x_{k-1} + b_k x_k + c_k x_{k+1} = d_k (Thomas algorithm:
 *     FORWARD elimination then BACKWARD substitution, Sec. 2.2).
 *   step: hdiff, then vadv with the diffused field as u_k.
 *   adjoints: transposes of the a.e. Jacobians with the limiter decisions of
 *     the forward pass held fixed (the mask), used by reverse-mode AD.
 *
 * A call follows the paper's statement of a stencil call (Sec. 2.2): fields,
 * read-only scalar parameters, and an iteration space given by a domain and
 * per-field origins; the vertical interval of a call is [0, nk) relative to
 * each field's origin; the horizontal halo is 2 (the stencil's radius).
 *
 * Conventions
 *   - All pointers in stencil_field.data, masks and workspaces are DEVICE
 *     pointers (hipMalloc'd or torch CUDA tensors).  Struct arguments
 *     themselves are host memory, read during the call only.
 *   - The caller owns every buffer.  The library never frees caller memory
 *     and never synchronises the device.  All compute calls are
 *     asynchronous on `stream` (NULL = the legacy default stream).
 *   - Errors: every int-returning call returns STENCIL_OK (0) or a negative
 *     STENCIL_E_* code; a message is kept in thread-local storage, read by
 *     stencil_last_error().  No exception crosses the ABI and nothing aborts.
 *     Argument validation reads host metadata only (O(1), no device access).
 *     Asynchronous kernel faults surface on a later call as STENCIL_E_HIP.
 *   - Outputs must not overlap inputs (an assignment is evaluated over the
 *     whole domain before it is stored, Sec. 2.2): STENCIL_E_ALIAS.
 */
#ifndef GT4MI_STENCIL_H
#define GT4MI_STENCIL_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STENCIL_ABI_VERSION 3
#define STENCIL_HALO 2

/* Element type.  The two range markers are not dtypes: they make every 32-bit
   value a value of the type, so that an unknown dtype passed by a caller is
   well defined in C++ and rejected with STENCIL_E_DTYPE. */
typedef enum {
  STENCIL_F32 = 0,
  STENCIL_F64 = 1,
  STENCIL_DTYPE_RANGE_MIN_ = -2147483647 - 1,
  STENCIL_DTYPE_RANGE_MAX_ = 2147483647
} stencil_dtype;

enum {
  STENCIL_OK = 0,
  STENCIL_E_NULL = -1,        /* a required pointer is NULL */
  STENCIL_E_DTYPE = -2,       /* unknown dtype, or misaligned data pointer */
  STENCIL_E_SHAPE = -3,       /* domain/origin/shape inconsistent */
  STENCIL_E_HALO = -4,        /* a field lacks the 2-point halo it needs */
  STENCIL_E_STRIDE = -5,      /* stride[0] != 1 or overlapping strides */
  STENCIL_E_ALIAS = -6,       /* an output overlaps an input */
  STENCIL_E_WORKSPACE = -7,   /* workspace missing or too small */
  STENCIL_E_UNSUPPORTED = -8, /* e.g. nk beyond the largest compiled class */
  STENCIL_E_HIP = -9,         /* a HIP runtime error (message attached) */
  STENCIL_E_ARG = -10         /* any other invalid argument */
};

/* A 3D field in device memory, index order (i, j, k), i fastest.
 *   data   : device pointer to allocation element (0,0,0)
 *   shape  : allocation extents in elements (i, j, k)
 *   stride : element strides; stride[0] must be 1; rows and planes must not
 *            overlap (stride[1] >= shape[0], stride[2] >= stride[1]*shape[1])
 *   origin : allocation index of compute-domain point (0,0,0)
 * Element (i,j,k) of the compute domain lives at
 *   data + (origin[0]+i) + (origin[1]+j)*stride[1] + (origin[2]+k)*stride[2].
 * Fields read with a halo need origin[0..1] >= 2 and
 * origin[d] + domain[d] + 2 <= shape[d] for d = 0, 1. */
typedef struct {
  void* data;
  int64_t shape[3];
  int64_t stride[3];
  int64_t origin[3];
} stencil_field;

typedef enum {
  STENCIL_IMPL_AUTO = 0,  /* fused kernels, tile from the tuning table */
  STENCIL_IMPL_FUSED = 1, /* all stages in one kernel, temporaries on chip */
  STENCIL_IMPL_PLAIN = 2  /* one kernel per stage, temporaries in HBM */
} stencil_impl;

typedef enum {
  STENCIL_COLUMN_AUTO = 0,
  STENCIL_COLUMN_REGISTERS = 1, /* one lane per column, its factors in VGPRs */
  STENCIL_COLUMN_OUTBUF = 2,    /* one lane per column, c' in VGPRs, d' staged in out */
  STENCIL_COLUMN_SPLIT = 3      /* two lanes per column eliminating from both ends,
                                   each holding half the factors in VGPRs (fused
                                   step: nk <= 160 in FP32; in FP64 nk <= 80, and
                                   nk <= 144 with f staged in out; longer columns
                                   take the one-ended solve) */
} stencil_column_store;

/* Boundary condition of a time step's output (the paper leaves halo
 * handling to the user; Sec. 2.2 only fixes that a stencil reads its halo). */
typedef enum {
  STENCIL_BOUNDARY_FROZEN = 0,  /* the output's halo is not written */
  STENCIL_BOUNDARY_PERIODIC = 1 /* after the step the output's 2-point halo holds
                                   the new interior at the wrapped indices
                                   (i mod ni, j mod nj), corners included */
} stencil_boundary;

/* Order in which the fused step's workgroups take their column tiles.  The
 * dispatcher hands consecutive workgroups to the 8 XCDs in turn, each with
 * its own L2; which order streams HBM faster depends on the tile shape and
 * the domain, so the autotuner measures both. */
typedef enum {
  STENCIL_ORDER_AUTO = 0,    /* tuned entry, else XCD */
  STENCIL_ORDER_XCD = 1,     /* each XCD takes one contiguous run of tiles,
                                so tiles sharing halo rows share an L2 */
  STENCIL_ORDER_DISPATCH = 2 /* workgroup t takes tile t: neighbouring tiles
                                run on different XCDs at the same time */
} stencil_tile_order;

/* Optional per-call options; pass NULL for defaults. */
/* Form of the horizontal diffusion's Laplacian stage (Sec. 3.1 names the
 * stencil; the workload's definition of it is the STATED form).  The DAMPING form
 * takes the discrete Laplacian itself, so that with every flux kept the
 * update is u - coeff * (discrete Laplacian applied twice), fourth-order
 * damping, where the stated form adds that term.  The limiter rule and the
 * update formula are the same in both; the limiter then keeps only fluxes
 * that run down the gradient of u. */
typedef enum {
  STENCIL_HDIFF_STATED = 0, /* lap = 4u - (u[i-1] + u[i+1] + u[j-1] + u[j+1]) */
  STENCIL_HDIFF_DAMPING = 1 /* lap = (u[i-1] + u[i+1] + u[j-1] + u[j+1]) - 4u */
} stencil_hdiff_form;

typedef struct {
  int32_t impl;         /* stencil_impl */
  int32_t tile_i;       /* horizontal tile of the fused forward kernels (step, */
  int32_t tile_j;       /*   batched step, hdiff of the generalised diffusion);
                           0 = tuned; supported: 64x4, 32x8, 16x16 (256
                           columns) and, for the two-ended step only (column
                           store SPLIT, else STENCIL_E_UNSUPPORTED), 64x2,
                           32x4, 16x8 (128 columns: 256-lane workgroups);
                           tile_j = 0 with tile_i set means the 256-column
                           tile.  FP64 columns of 97..144 levels in the
                           two-ended step run tile_i x (128 / tile_i) tiles.
                           Other calls use the tile's width only; the stated
                           hdiff and the adjoints' gather walk fixed strips
                           and ignore it (the value is still validated). */
  int32_t column_store; /* stencil_column_store */
  void* workspace;      /* device memory for STENCIL_IMPL_PLAIN temporaries */
  size_t workspace_bytes;
  int32_t boundary;     /* stencil_boundary of stencil_step (and of the graph
                           loop, which calls it): PERIODIC needs an output
                           with the 2-point halo */
  /* The generalised horizontal diffusion (stencil_hdiff, stencil_step, the
   * graph loop and their adjoints; fused kernels only, the step with
   * nk <= 144 in FP64 / 160 in FP32; PLAIN, the batched calls and longer
   * columns return STENCIL_E_UNSUPPORTED).  Zero-initialised options keep
   * the stated form with the scalar coefficient. */
  int32_t hdiff_form;               /* stencil_hdiff_form */
  const stencil_field* coeff_field; /* NULL: the scalar coeff argument.  Else a
                                       per-point coefficient kappa(i,j,k) on the
                                       domain (interior layout, like data) that
                                       replaces it in the update, out = u -
                                       kappa * div; the scalar is then ignored
                                       (the adjoints take their coefficient
                                       from here too).  Read, never written. */
  int32_t tile_order; /* stencil_tile_order of the fused step (two-ended
                         column store); other kernels ignore it */
} stencil_options;

typedef enum {
  STENCIL_OP_HDIFF = 0,
  STENCIL_OP_VADV = 1,
  STENCIL_OP_STEP = 2,
  STENCIL_OP_HDIFF_ADJOINT = 3,
  STENCIL_OP_VADV_ADJOINT = 4,
  STENCIL_OP_STEP_ADJOINT = 5
} stencil_op;

/* ---------------------------------------------------------------- info */
/* ABI version (STENCIL_ABI_VERSION). */
int stencil_version(void);
/* Message of the last failed call on this thread ("" if none). */
const char* stencil_last_error(void);
/* Largest nk the fused column kernels accept (longer columns: PLAIN). */
int stencil_max_fused_nk(stencil_dtype dtype);

/* Bytes of the limiter mask of a domain (device buffer, caller-owned).
 * Layout, for W = ceil(ni/64) 64-bit words per row, all sections 256-byte
 * aligned, bit b of a word = i = 64*word + b, 1 = flux kept:
 *   X plane  uint64[nk][nj][W] : flux between (i,j) and (i+1,j), i in [0,ni)
 *   Y plane  uint64[nk][nj][W] : flux between (i,j) and (i,j+1), i in [0,ni)
 *   X edge   uint8 [nk][nj]    : flux between (-1,j) and (0,j)
 *   Y edge   uint8 [nk][ni]    : flux between (i,-1) and (i,0)
 * Returns 0 for an invalid domain. */
size_t stencil_mask_bytes(const int64_t domain[3]);

/* Device workspace needed by `op` under `opts` (0 if none).  PLAIN forms
 * keep their stage temporaries there; STEP_ADJOINT without a data_bar
 * output keeps the column adjoint there. */
size_t stencil_workspace_bytes(int op, stencil_dtype dtype, const int64_t domain[3],
                               const stencil_options* opts);

/* ------------------------------------------------------------- forward */
/* Horizontal diffusion (named in Sec. 3.1; formulas above).  u: read on the domain plus a 2-point
 * halo in i and j.  out: the interior is written, its halo is untouched.
 * mask: NULL, or stencil_mask_bytes(domain) device bytes that receive the
 * limiter decisions.  opts->hdiff_form and opts->coeff_field select the
 * generalised diffusion (the coefficient field may not overlap out). */
int stencil_hdiff(stencil_dtype dtype, const stencil_field* u, stencil_field* out,
                  const int64_t domain[3], double coeff, void* mask,
                  const stencil_options* opts, hipStream_t stream);

/* Vertical advection (named in Sec. 3.1; formulas above): out = T(w)^{-1} (u + data) per column.
 * u, data: domain; w: nk+1 staggered levels (w_0 and w_nk are not read);
 * out: domain (interior only). */
int stencil_vadv(stencil_dtype dtype, const stencil_field* u, const stencil_field* data,
                 const stencil_field* w, stencil_field* out, const int64_t domain[3],
                 double dt_dz, const stencil_options* opts, hipStream_t stream);

/* One time step: out = vadv(hdiff(u), data, w).  Arguments as above; the
 * halo of out is untouched (ping-pong buffers with equal halos keep a
 * frozen boundary) unless opts->boundary is PERIODIC, which then fills it
 * from the new interior.  The diffusion follows opts->hdiff_form and
 * opts->coeff_field as in stencil_hdiff. */
int stencil_step(stencil_dtype dtype, const stencil_field* u, const stencil_field* data,
                 const stencil_field* w, stencil_field* out, const int64_t domain[3],
                 double coeff, double dt_dz, void* mask, const stencil_options* opts,
                 hipStream_t stream);

/* ------------------------------------------------------------- adjoint */
/* u_bar = J_hdiff^T out_bar with the forward limiter mask held fixed.
 * out_bar: domain.  u_bar: written over the domain plus its 2-point halo
 * (every padded point is overwritten, the corner points never read by the
 * forward stencil receive 0).  mask: from a forward call on this domain
 * with the same opts->hdiff_form; opts->coeff_field, when set, is the
 * forward's per-point coefficient. */
int stencil_hdiff_adjoint(stencil_dtype dtype, const stencil_field* out_bar, const void* mask,
                          stencil_field* u_bar, const int64_t domain[3], double coeff,
                          const stencil_options* opts, hipStream_t stream);

/* d_bar = T(w)^{-T} x_bar per column, coefficients recomputed from w. */
int stencil_vadv_adjoint(stencil_dtype dtype, const stencil_field* x_bar,
                         const stencil_field* w, stencil_field* d_bar,
                         const int64_t domain[3], double dt_dz, const stencil_options* opts,
                         hipStream_t stream);

/* Adjoint of stencil_step: lambda = T^{-T} x_bar; u_bar = J_hdiff^T lambda
 * (domain plus halo); data_bar = lambda if data_bar is not NULL (else the
 * workspace of opts holds lambda, stencil_workspace_bytes(STEP_ADJOINT)).
 * opts->hdiff_form and opts->coeff_field as for stencil_hdiff_adjoint. */
int stencil_step_adjoint(stencil_dtype dtype, const stencil_field* x_bar,
                         const stencil_field* w, const void* mask, stencil_field* u_bar,
                         stencil_field* data_bar, const int64_t domain[3], double coeff,
                         double dt_dz, const stencil_options* opts, hipStream_t stream);

/* Fill the 2-point halo of `f` (a field with the halo, as u) on `domain`
 * according to `boundary`: PERIODIC copies the interior at the wrapped
 * indices, corners included (the single-GPU half of a halo exchange);
 * FROZEN does nothing.  The interior is not modified. */
int stencil_halo_update(stencil_dtype dtype, stencil_field* f, const int64_t domain[3], int boundary,
                        hipStream_t stream);

/* ------------------------------------------------------ parameter gradients */
/* Gradients of a scalar loss L with respect to the parameters of one step
 * (parameter tuning).  With the limiter decisions held fixed the diffusion
 * is h = u - coeff D(u), D the divergence of the limited fluxes (it does not
 * depend on coeff), and the column solve is T(w) x = h + data.  With x_bar
 * = dL/dx, lam = T^{-T} x_bar (the data_bar output of stencil_step_adjoint)
 * and x the step's output:
 *   coeff_bar = -sum over the domain of lam * D(u)
 *   w_bar_j   = r/4 [lam_j x_{j-1} - lam_{j-1} x_j - s_j (lam_j x_j + lam_{j-1} x_{j-1})]
 * for j = 1 .. nk-1, r = dt_dz, s_j = sign w_j (0 at 0: the a.e. derivative
 * of |a|, |c| in b); w_bar_0 = w_bar_nk = 0 (those levels do not enter T).
 *   u: the step's input (domain plus 2-point halo); lam, x: domain;
 *   w, w_bar: nk+1 staggered levels (w_bar written on all of them);
 *   coeff_bar: device pointer to one double (FP64 for both dtypes; the
 *     per-point products are summed in FP64 per 64 x 4 tile, then over the
 *     tiles in a fixed order, so the result is reproducible).
 * Either output may be NULL (not both).  coeff_bar needs a device
 * workspace of stencil_param_workspace_bytes(domain) bytes (8-byte aligned)
 * for the per-tile sums.  Outputs may not overlap inputs, the workspace or
 * each other (STENCIL_E_ALIAS).  opts (NULL: defaults): hdiff_form selects
 * the D of coeff_bar; a forward with opts->coeff_field has no scalar
 * coefficient, so coeff_bar must then be NULL (STENCIL_E_ARG; its gradient
 * is stencil_coeff_field_adjoint's). */
size_t stencil_param_workspace_bytes(stencil_dtype dtype, const int64_t domain[3]);
int stencil_step_param_adjoint(stencil_dtype dtype, const stencil_field* u, const stencil_field* w,
                               const stencil_field* x, const stencil_field* lam,
                               stencil_field* w_bar, double* coeff_bar, const int64_t domain[3],
                               double dt_dz, const stencil_options* opts, void* ws, size_t ws_bytes,
                               hipStream_t stream);

/* Gradient with respect to the per-point coefficient of the generalised
 * diffusion: out(p) depends on kappa(p) only through -kappa(p) D(u)(p), so
 *   kappa_bar(p) = -lam(p) D(u)(p)
 * with D for opts->hdiff_form (NULL opts: the stated form) and lam the
 * cotangent of the diffusion's output: out_bar for stencil_hdiff, the
 * data_bar of stencil_step_adjoint for a step.  u: the forward input
 * (domain plus 2-point halo); lam, kappa_bar: domain.  kappa_bar may not
 * overlap u or lam (STENCIL_E_ALIAS).  The limiter decisions are recomputed
 * from u, as the forward took them. */
int stencil_coeff_field_adjoint(stencil_dtype dtype, const stencil_field* u, const stencil_field* lam,
                                stencil_field* kappa_bar, const int64_t domain[3],
                                const stencil_options* opts, hipStream_t stream);

/* ------------------------------------------------------------- batched */
/* Many independent fields of uneven sizes in one persistent launch (each
 * field is its own stencil call in the sense of Sec. 2.2; the batch only
 * shares the launch).  Every item obeys the rules of the single-field call
 * it stands for, and additionally no output of one item may overlap any
 * buffer of another (all items run concurrently): STENCIL_E_ALIAS.
 * Limits: n <= 1024 items, nk <= 144 per item (STENCIL_E_UNSUPPORTED), the
 * fused kernels only (impl PLAIN, or a PERIODIC boundary: STENCIL_E_UNSUPPORTED).  Items with an
 * empty domain are skipped (their outputs untouched), except that an
 * adjoint item with nk > 0 and an empty horizontal domain zeroes u_bar as
 * the single-field adjoint does.  The forward's tile is opts->tile_i, else
 * the tuning table's entry for the batch's largest field. */

/* One field of a batch: forward step out = step(u, data, w) on `domain`. */
typedef struct {
  stencil_field u, data, w, out;
  int64_t domain[3];
  double coeff, dt_dz;
  void* mask; /* NULL or stencil_mask_bytes(domain) bytes */
} stencil_batch_item;

/* One field of an adjoint batch (arguments of stencil_step_adjoint). */
typedef struct {
  stencil_field x_bar, w, u_bar, data_bar; /* data_bar.data may be NULL */
  int64_t domain[3];
  double coeff, dt_dz;
  const void* mask;
} stencil_batch_adjoint_item;

/* Device workspace of a batch (0 for n <= 0, an invalid dtype, or a batch
 * with no work): the work list (a header, per-field prefix sums of work
 * items and the argument blocks of the fields, rewritten by every call) and,
 * for the adjoint, lambda = T^{-T} x_bar of every item without data_bar. */
size_t stencil_batch_workspace_bytes(stencil_dtype dtype, int n, const stencil_batch_item* items);
size_t stencil_batch_adjoint_workspace_bytes(stencil_dtype dtype, int n,
                                             const stencil_batch_adjoint_item* items);

/* All n steps in one persistent launch (FP64: two, one for the fields with
 * columns of up to 80 levels, one for the longer ones, which run tiles of
 * tile_i x (128 / tile_i) columns).  opts->tile_i, when set, is the tile of
 * every field; when 0 each field takes its size class's tuned tile, or
 * without one the width (64, 32 or 16) that leaves the fewest lanes idle
 * on its ragged edges.  The call sorts the items longest
 * column first, writes the work list into `ws` with small copy kernels on
 * `stream` (stream-ordered, so the call can be captured into a graph), and
 * launches the kernel(s), whose workgroups pull (field, tile) work items from a
 * device counter in `ws` until none are left.  ws: device memory, 256-byte
 * aligned, at least stencil_batch_workspace_bytes(...) bytes, not
 * overlapping any field (STENCIL_E_WORKSPACE / STENCIL_E_ALIAS); two calls
 * that may run at the same time need distinct workspaces. */
int stencil_step_batched(stencil_dtype dtype, int n, const stencil_batch_item* items, void* ws,
                         size_t ws_bytes, const stencil_options* opts, hipStream_t stream);
/* The adjoints of a batch: one persistent launch for the column adjoints
 * (work items: field, 64x4 column tile), then one launch for the horizontal
 * gathers with a workgroup per work item (field, four strips of the padded
 * domain, level; a strip is 60 x 8 points in FP64, 124 x 12 in FP32).  ws as for the forward, sized by
 * stencil_batch_adjoint_workspace_bytes; opts->tile_i is not used. */
int stencil_step_adjoint_batched(stencil_dtype dtype, int n,
                                 const stencil_batch_adjoint_item* items, void* ws,
                                 size_t ws_bytes, const stencil_options* opts,
                                 hipStream_t stream);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * forward batch of stencil_step_batched with its work list in a fixed
 * device array of STENCIL_NOALLOC_SCRATCH_BYTES bytes that the library
 * holds on each device it runs on until the process ends, instead of a
 * caller workspace.  The call allocates no device memory.  Arguments,
 * validation, results (bit for bit) and limits are those of
 * stencil_step_batched; a batch whose work list
 * (stencil_batch_workspace_bytes) is larger than the array is refused with
 * STENCIL_E_UNSUPPORTED (any batch of up to 256 fields fits).  Every call
 * on a device uses that device's one array: calls that may run at the same
 * time on one device (two streams, two threads, two graphs) race, and the
 * caller must order them. */
#define STENCIL_NOALLOC_SCRATCH_BYTES 65536
int stencil_step_batched_noalloc(stencil_dtype dtype, int n, const stencil_batch_item* items,
                                 const stencil_options* opts, hipStream_t stream);

/* ---------------------------------------------------------- hipGraph loop */
typedef struct stencil_graph stencil_graph;

/* Captures nsteps stencil_step calls into a HIP graph: step s reads the
 * buffer it did not write at step s-1 (u_a -> u_b -> u_a ...), so after the
 * graph runs the state is in u_b for odd nsteps and in u_a for even.  Both
 * buffers must hold the same halo.  `stream` is used for capture only. */
int stencil_graph_capture_steps(stencil_dtype dtype, int nsteps, stencil_field* u_a,
                                stencil_field* u_b, const stencil_field* data,
                                const stencil_field* w, const int64_t domain[3], double coeff,
                                double dt_dz, const stencil_options* opts, hipStream_t stream,
                                stencil_graph** graph);
int stencil_graph_launch(stencil_graph* graph, hipStream_t stream);
int stencil_graph_destroy(stencil_graph* graph);

/* ---------------------------------------------------------------- tuning */
/* Times every tile candidate of `op` (STENCIL_OP_STEP: tile x column store,
 * and for the two-ended column store both workgroup sizes (256- and
 * 128-column tiles) and both tile orders; or STENCIL_OP_HDIFF,
 * timed in the damping form: only the generalised diffusion's hdiff has a
 * tile; the other ops have none to choose: STENCIL_E_ARG) on a domain of this size (scratch
 * fields allocated and freed by the library for the duration of the call,
 * device synchronised) and records the fastest in the process-wide tuning
 * table under (dtype, op, size class).  *best_us receives its time. */
int stencil_autotune(stencil_dtype dtype, int op, const int64_t domain[3], int reps,
                     double* best_us);
/* The step's candidates timed on the caller's own fields, on `stream` (which
 * is synchronised before the call returns): which tile and tile order stream
 * HBM fastest depends on where the fields sit in memory as well as on their
 * shape, so tuning on the storages a time loop will use measures what it
 * will run.  op must be STENCIL_OP_STEP (else STENCIL_E_ARG); the fields obey
 * stencil_step's rules; `out` is overwritten (its interior), the inputs are
 * only read.  Records the fastest candidate under (dtype, op, size class) as
 * stencil_autotune does. */
int stencil_autotune_fields(stencil_dtype dtype, int op, const stencil_field* u,
                            const stencil_field* data, const stencil_field* w, stencil_field* out,
                            const int64_t domain[3], int reps, hipStream_t stream, double* best_us);
/* Tile, column store and tile order chosen for (dtype, op, domain) -- the
 * tuned entry or the default.  tile_order may be NULL. */
int stencil_tuning_lookup(stencil_dtype dtype, int op, const int64_t domain[3], int32_t* tile_i,
                          int32_t* tile_j, int32_t* column_store, int32_t* tile_order);
/* Persist / restore the tuning table as JSON. */
int stencil_save_tuning(const char* json_path);
int stencil_load_tuning(const char* json_path);
int stencil_clear_tuning(void);

#ifdef __cplusplus
}
#endif
#endif /* GT4MI_STENCIL_H */
