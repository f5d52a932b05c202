/*
 * oracle.c -- plain, slow, obviously-correct FP64 CPU reference for the
 * stencil hot path (horizontal diffusion, implicit vertical advection, their
 * time step and the hand-derived adjoints).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or table with the HIP
 * library.
 *
 * Sources:
 *   - Semantics of a stencil call (GT4Py paper, Sec. 2.2): the horizontal
 *     plane is always parallel; vertical computations run PARALLEL, FORWARD
 *     or BACKWARD; intervals specialise boundary levels; an assignment is
 *     evaluated over the whole domain before it is stored (so the output
 *     never aliases the input); temporaries are not observable; the
 *     iteration space comes from domain/origin.
 *   - The two benchmark stencils the paper names in Sec. 3.1: the
 *     multi-stage horizontal diffusion and the vertical advection implicit
 *     solver.  The paper prints no formula for either; the formulas below
 *     are the benchmark workload's definition of the two stencils, taken
 *     literally:
 *       lap  = 4u - u[i-1] - u[i+1] - u[j-1] - u[j+1]
 *       flx  = lap[i+1] - lap[i], zeroed where flx * (u[i+1]-u[i]) > 0
 *       fly  = the same along j
 *       out  = u - coeff * (flx - flx[i-1] + fly - fly[j-1])
 *     and, per column with r = dt/dz,
 *       a_k = -r/4 * w_k (k >= 1),  c_k = +r/4 * w_{k+1} (k <= nk-2),
 *       a_0 = c_{nk-1} = 0,  b_k = 1 + |a_k| + |c_k|,  d_k = u_k + data_k,
 *     solved by the Thomas algorithm (FORWARD elimination, BACKWARD
 *     substitution).
 *   - Two generalisations of the diffusion, parity unaffected for the
 *     stated form: a per-point coefficient kappa(i,j,k) in place of the
 *     scalar coeff in the update, and a damping form whose Laplacian stage
 *     is the discrete Laplacian itself (the negative of the stated lap),
 *     every later stage unchanged.  With every flux kept the stated form
 *     adds coeff times the squared discrete Laplacian, the damping form
 *     subtracts it (fourth-order diffusion).
 *
 * Array conventions (C order, all strides implied by the sizes):
 *   padded  u, out, ubar : [nk][nj+4][ni+4], U(i,j,k) = u[k][j+2][i+2],
 *                          i in [-2, ni+2), j in [-2, nj+2)
 *   interior data, x, lam, xbar : [nk][nj][ni]
 *   staggered w          : [nk+1][nj][ni]
 *   masks (1 = flux kept, 0 = limiter zeroed it)
 *     mx : [nk][nj][ni+1],  MX(i,j,k) = mx[k][j][i+1], i in [-1, ni)
 *          flux between (i,j) and (i+1,j)
 *     my : [nk][nj+1][ni],  MY(i,j,k) = my[k][j+1][i], j in [-1, nj)
 *          flux between (i,j) and (i,j+1)
 *
 * Limiter decision precision: `decide_f32 == 0` takes the limiter decision in
 * FP64; `decide_f32 != 0` computes lap, the flux difference and the gradient
 * used *for the decision only* in IEEE binary32 with the same association,
 * so that a binary32 implementation and this reference branch identically.
 * All values are always carried in FP64.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC; a second
 * build adds -fopenmp for the CPU baseline on all host cores.  Its parallel
 * regions split independent levels (horizontal stages) or independent
 * columns (the tridiagonal solves) over threads, each with its own
 * temporaries, so every value is computed by the same operations in the
 * same order and both builds give identical results.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* indexing helpers                                                     */
/* ------------------------------------------------------------------ */
#define PAD 2
#define UIDX(i, j, k) ((size_t)(k) * (size_t)(nj + 2 * PAD) * (size_t)(ni + 2 * PAD) + \
                       (size_t)((j) + PAD) * (size_t)(ni + 2 * PAD) + (size_t)((i) + PAD))
#define IIDX(i, j, k) ((size_t)(k) * (size_t)nj * (size_t)ni + (size_t)(j) * (size_t)ni + (size_t)(i))
#define MXIDX(i, j, k) ((size_t)(k) * (size_t)nj * (size_t)(ni + 1) + (size_t)(j) * (size_t)(ni + 1) + (size_t)((i) + 1))
#define MYIDX(i, j, k) ((size_t)(k) * (size_t)(nj + 1) * (size_t)ni + (size_t)((j) + 1) * (size_t)ni + (size_t)(i))

/* The limiter (the workload's definition of the diffusion): the flux is zeroed where
 * flux * gradient > 0, the product taken literally in the precision of the
 * decision (binary64, or binary32 when decide_f32 is set). */
static int limiter_keeps(double f, double g) { return !(f * g > 0.0); }
static int limiter_keeps_f32(float f, float g) { return !(f * g > 0.0f); }

/* Laplacian stage, fixed association.  The stated form takes
 * 4u - ((u[i-1]+u[i+1]) + (u[j-1]+u[j+1])), the negative of the discrete
 * Laplacian; the damping form (`damping` != 0) takes the discrete Laplacian
 * itself, ((u[i-1]+u[i+1]) + (u[j-1]+u[j+1])) - 4u, with every later stage
 * unchanged, so that with every flux kept the update is u - coeff * (discrete
 * Laplacian applied twice): fourth-order damping. */
static double lap64(const double* u, int ni, int nj, int i, int j, int k, int damping) {
  double s = (u[UIDX(i - 1, j, k)] + u[UIDX(i + 1, j, k)]) +
             (u[UIDX(i, j - 1, k)] + u[UIDX(i, j + 1, k)]);
  double c = 4.0 * u[UIDX(i, j, k)];
  return damping ? s - c : c - s;
}
static float lap32(const double* u, int ni, int nj, int i, int j, int k, int damping) {
  float s = ((float)u[UIDX(i - 1, j, k)] + (float)u[UIDX(i + 1, j, k)]) +
            ((float)u[UIDX(i, j - 1, k)] + (float)u[UIDX(i, j + 1, k)]);
  float c = 4.0f * (float)u[UIDX(i, j, k)];
  return damping ? s - c : c - s;
}

/* ------------------------------------------------------------------ */
/* Limiter masks of the horizontal diffusion (workload definition)       */
/* ------------------------------------------------------------------ */
void oracle_hdiff_masks_form(int ni, int nj, int nk, const double* u, int decide_f32, int damping,
                             unsigned char* mx, unsigned char* my) {
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nk; ++k) {
    /* x-fluxes on [-1, ni) x [0, nj) */
    for (int j = 0; j < nj; ++j)
      for (int i = -1; i < ni; ++i) {
        int keep;
        if (decide_f32) {
          float f = lap32(u, ni, nj, i + 1, j, k, damping) - lap32(u, ni, nj, i, j, k, damping);
          float g = (float)u[UIDX(i + 1, j, k)] - (float)u[UIDX(i, j, k)];
          keep = limiter_keeps_f32(f, g);
        } else {
          double f = lap64(u, ni, nj, i + 1, j, k, damping) - lap64(u, ni, nj, i, j, k, damping);
          double g = u[UIDX(i + 1, j, k)] - u[UIDX(i, j, k)];
          keep = limiter_keeps(f, g);
        }
        mx[MXIDX(i, j, k)] = (unsigned char)keep;
      }
    /* y-fluxes on [0, ni) x [-1, nj) */
    for (int j = -1; j < nj; ++j)
      for (int i = 0; i < ni; ++i) {
        int keep;
        if (decide_f32) {
          float f = lap32(u, ni, nj, i, j + 1, k, damping) - lap32(u, ni, nj, i, j, k, damping);
          float g = (float)u[UIDX(i, j + 1, k)] - (float)u[UIDX(i, j, k)];
          keep = limiter_keeps_f32(f, g);
        } else {
          double f = lap64(u, ni, nj, i, j + 1, k, damping) - lap64(u, ni, nj, i, j, k, damping);
          double g = u[UIDX(i, j + 1, k)] - u[UIDX(i, j, k)];
          keep = limiter_keeps(f, g);
        }
        my[MYIDX(i, j, k)] = (unsigned char)keep;
      }
  }
}

void oracle_hdiff_masks(int ni, int nj, int nk, const double* u, int decide_f32,
                        unsigned char* mx, unsigned char* my) {
  oracle_hdiff_masks_form(ni, nj, nk, u, decide_f32, 0, mx, my);
}

/* ------------------------------------------------------------------ */
/* Horizontal diffusion with the limiter masks given: the four stages   */
/* lap -> flx -> fly -> out, evaluated stage by stage over the whole    */
/* level (Sec. 2.2: each assignment covers the full domain first).      */
/* With masks taken from the same u this is the forward stencil; with   */
/* masks held fixed it is its (a.e.) tangent-linear map.                */
/* Writes the interior of `out` only (out[k][j][i], interior layout).   */
/* ------------------------------------------------------------------ */
/* The coefficient of the update at interior point (i,j,k): the scalar
 * coeff, or the per-point field kappa (interior layout) when given. */
#define COEF(i, j, k) (kappa ? kappa[IIDX(i, j, k)] : coeff)

static void hdiff_with_masks(int ni, int nj, int nk, const double* u, double coeff,
                             const double* kappa, int damping, const unsigned char* mx,
                             const unsigned char* my, double* out_interior) {
  const int li = ni + 2, lj = nj + 2; /* lap on the box [-1,ni] x [-1,nj] */
#pragma omp parallel
  { /* levels are independent: one set of level temporaries per thread */
  double* lap = (double*)malloc(sizeof(double) * (size_t)li * (size_t)lj);
  double* fx = (double*)malloc(sizeof(double) * (size_t)(ni + 1) * (size_t)nj);
  double* fy = (double*)malloc(sizeof(double) * (size_t)ni * (size_t)(nj + 1));
#define LAP(i, j) lap[(size_t)((j) + 1) * (size_t)li + (size_t)((i) + 1)]
#define FX(i, j) fx[(size_t)(j) * (size_t)(ni + 1) + (size_t)((i) + 1)]
#define FY(i, j) fy[(size_t)((j) + 1) * (size_t)ni + (size_t)(i)]
#pragma omp for schedule(static)
  for (int k = 0; k < nk; ++k) {
    for (int j = -1; j <= nj; ++j)
      for (int i = -1; i <= ni; ++i) LAP(i, j) = lap64(u, ni, nj, i, j, k, damping);
    for (int j = 0; j < nj; ++j)
      for (int i = -1; i < ni; ++i) {
        double f = LAP(i + 1, j) - LAP(i, j);
        FX(i, j) = mx[MXIDX(i, j, k)] ? f : 0.0;
      }
    for (int j = -1; j < nj; ++j)
      for (int i = 0; i < ni; ++i) {
        double f = LAP(i, j + 1) - LAP(i, j);
        FY(i, j) = my[MYIDX(i, j, k)] ? f : 0.0;
      }
    for (int j = 0; j < nj; ++j)
      for (int i = 0; i < ni; ++i) {
        double div = (FX(i, j) - FX(i - 1, j)) + (FY(i, j) - FY(i, j - 1));
        out_interior[IIDX(i, j, k)] = u[UIDX(i, j, k)] - COEF(i, j, k) * div;
      }
  }
#undef LAP
#undef FX
#undef FY
  free(lap);
  free(fx);
  free(fy);
  }
}

/* Forward horizontal diffusion, general form: per-point coefficient kappa
 * (NULL: the scalar coeff) and the damping form of the Laplacian.  `out` is
 * padded: interior = the update, halo = a copy of u's halo (the halo is
 * never computed, only carried). */
void oracle_hdiff_gen(int ni, int nj, int nk, const double* u, double coeff, const double* kappa,
                      int damping, int decide_f32, double* out, unsigned char* mx,
                      unsigned char* my) {
  oracle_hdiff_masks_form(ni, nj, nk, u, decide_f32, damping, mx, my);
  double* h = (double*)malloc(sizeof(double) * (size_t)ni * (size_t)nj * (size_t)nk + 8);
  hdiff_with_masks(ni, nj, nk, u, coeff, kappa, damping, mx, my, h);
  memcpy(out, u, sizeof(double) * (size_t)(ni + 4) * (size_t)(nj + 4) * (size_t)nk);
  for (int k = 0; k < nk; ++k)
    for (int j = 0; j < nj; ++j)
      for (int i = 0; i < ni; ++i) out[UIDX(i, j, k)] = h[IIDX(i, j, k)];
  free(h);
}

/* The stated form with a scalar coefficient. */
void oracle_hdiff(int ni, int nj, int nk, const double* u, double coeff, int decide_f32,
                  double* out, unsigned char* mx, unsigned char* my) {
  oracle_hdiff_gen(ni, nj, nk, u, coeff, NULL, 0, decide_f32, out, mx, my);
}

/* ------------------------------------------------------------------ */
/* Vertical advection (workload definition): tridiagonal system per     */
/* column; the boundary rows (intervals, Sec. 2.2) have a_0 = 0 and     */
/* c_{nk-1} = 0.  Thomas algorithm: FORWARD elimination then BACKWARD   */
/* substitution (Sec. 2.2 vertical iteration orders).                   */
/* ------------------------------------------------------------------ */
static double coef_a(const double* w, int ni, int nj, int i, int j, int k, double r) {
  (void)nj;
  return k >= 1 ? (-0.25 * r) * w[(size_t)k * (size_t)nj * (size_t)ni + (size_t)j * (size_t)ni + (size_t)i] : 0.0;
}
static double coef_c(const double* w, int ni, int nj, int nk, int i, int j, int k, double r) {
  return k <= nk - 2 ? (0.25 * r) * w[(size_t)(k + 1) * (size_t)nj * (size_t)ni + (size_t)j * (size_t)ni + (size_t)i] : 0.0;
}

/* x = T^{-1} d per column, d[k] given (interior layout). */
static void thomas_columns(int ni, int nj, int nk, const double* d, const double* w, double dt_dz,
                           double* x) {
#pragma omp parallel
  { /* columns are independent: one pair of column temporaries per thread */
  double* cp = (double*)malloc(sizeof(double) * (size_t)nk + 8);
  double* dp = (double*)malloc(sizeof(double) * (size_t)nk + 8);
#pragma omp for schedule(static)
  for (int j = 0; j < nj; ++j)
    for (int i = 0; i < ni; ++i) {
      for (int k = 0; k < nk; ++k) {
        double a = coef_a(w, ni, nj, i, j, k, dt_dz);
        double c = coef_c(w, ni, nj, nk, i, j, k, dt_dz);
        double b = 1.0 + fabs(a) + fabs(c);
        double dk = d[IIDX(i, j, k)];
        if (k == 0) {
          cp[0] = c / b;
          dp[0] = dk / b;
        } else {
          double m = b - a * cp[k - 1];
          cp[k] = c / m;
          dp[k] = (dk - a * dp[k - 1]) / m;
        }
      }
      x[IIDX(i, j, nk - 1)] = dp[nk - 1];
      for (int k = nk - 2; k >= 0; --k) x[IIDX(i, j, k)] = dp[k] - cp[k] * x[IIDX(i, j, k + 1)];
    }
  free(cp);
  free(dp);
  }
}

/* vadv alone: right-hand side d = u_in + data, all interior layout. */
void oracle_vadv(int ni, int nj, int nk, const double* uin, const double* data, const double* w,
                 double dt_dz, double* x) {
  if (ni <= 0 || nj <= 0 || nk <= 0) return;
  size_t n = (size_t)ni * (size_t)nj * (size_t)nk;
  double* d = (double*)malloc(sizeof(double) * n);
  for (size_t p = 0; p < n; ++p) d[p] = uin[p] + data[p];
  thomas_columns(ni, nj, nk, d, w, dt_dz, x);
  free(d);
}

/* One time step: horizontal diffusion (general form), then vertical
 * advection with the diffused field as u_k in d_k = u_k + data_k.  `next` is
 * padded: interior = x, halo = u's halo (held fixed). */
void oracle_step_gen(int ni, int nj, int nk, const double* u, const double* data, const double* w,
                     double coeff, const double* kappa, int damping, double dt_dz, int decide_f32,
                     double* next, unsigned char* mx, unsigned char* my) {
  size_t n = (size_t)ni * (size_t)nj * (size_t)nk;
  memcpy(next, u, sizeof(double) * (size_t)(ni + 4) * (size_t)(nj + 4) * (size_t)nk);
  if (n == 0) return;
  oracle_hdiff_masks_form(ni, nj, nk, u, decide_f32, damping, mx, my);
  double* h = (double*)malloc(sizeof(double) * n);
  double* x = (double*)malloc(sizeof(double) * n);
  hdiff_with_masks(ni, nj, nk, u, coeff, kappa, damping, mx, my, h);
#pragma omp parallel for schedule(static)
  for (size_t p = 0; p < n; ++p) h[p] += data[p];
  thomas_columns(ni, nj, nk, h, w, dt_dz, x);
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nk; ++k)
    for (int j = 0; j < nj; ++j)
      for (int i = 0; i < ni; ++i) next[UIDX(i, j, k)] = x[IIDX(i, j, k)];
  free(h);
  free(x);
}

void oracle_step(int ni, int nj, int nk, const double* u, const double* data, const double* w,
                 double coeff, double dt_dz, int decide_f32, double* next, unsigned char* mx,
                 unsigned char* my) {
  oracle_step_gen(ni, nj, nk, u, data, w, coeff, NULL, 0, dt_dz, decide_f32, next, mx, my);
}

/* ------------------------------------------------------------------ */
/* Adjoints (transpose of the a.e. Jacobian, limiter masks held fixed)  */
/* ------------------------------------------------------------------ */

/* Horizontal diffusion adjoint: ubar = J_h^T lam over the whole padded
 * domain, general form.  lam is given on the interior and is zero outside
 * it. */
void oracle_hdiff_adjoint_gen(int ni, int nj, int nk, const double* lam, const unsigned char* mx,
                              const unsigned char* my, double coeff, const double* kappa,
                              int damping, double* ubar) {
  const int li = ni + 2, lj = nj + 2;
#pragma omp parallel
  { /* levels are independent: one set of level temporaries per thread */
  double* gx = (double*)malloc(sizeof(double) * (size_t)(ni + 1) * (size_t)(nj > 0 ? nj : 1));
  double* gy = (double*)malloc(sizeof(double) * (size_t)(ni > 0 ? ni : 1) * (size_t)(nj + 1));
  double* lb = (double*)malloc(sizeof(double) * (size_t)li * (size_t)lj);
#define INI(i, j) ((i) >= 0 && (i) < ni && (j) >= 0 && (j) < nj)
#define LAM(i, j) (INI(i, j) ? lam[IIDX(i, j, k)] : 0.0)
#define MU(i, j) (INI(i, j) ? kappa[IIDX(i, j, k)] * lam[IIDX(i, j, k)] : 0.0)
#define GX(i, j) ((((i) >= -1 && (i) < ni && (j) >= 0 && (j) < nj)) ? gx[(size_t)(j) * (size_t)(ni + 1) + (size_t)((i) + 1)] : 0.0)
#define GY(i, j) ((((i) >= 0 && (i) < ni && (j) >= -1 && (j) < nj)) ? gy[(size_t)((j) + 1) * (size_t)ni + (size_t)(i)] : 0.0)
#define LB(i, j) ((((i) >= -1 && (i) <= ni && (j) >= -1 && (j) <= nj)) ? lb[(size_t)((j) + 1) * (size_t)li + (size_t)((i) + 1)] : 0.0)
#pragma omp for schedule(static)
  for (int k = 0; k < nk; ++k) {
    /* out(p) = u(p) - coeff(p) * (Fx(p) - Fx(p-ei) + Fy(p) - Fy(p-ej)):
     * dout(p)/dFx(q) = -coeff(p) if q == p, +coeff(p) if q == p - ei, so
     * Fx(q) collects -(coeff lam)(q) + (coeff lam)(q+ei).
     * Fx(q) = MX(q) * (lap(q+ei) - lap(q)). Keep the masked flux cotangent. */
    for (int j = 0; j < nj; ++j)
      for (int i = -1; i < ni; ++i) {
        double fbar = kappa ? -(MU(i, j) - MU(i + 1, j)) : -coeff * (LAM(i, j) - LAM(i + 1, j));
        gx[(size_t)j * (size_t)(ni + 1) + (size_t)(i + 1)] = mx[MXIDX(i, j, k)] ? fbar : 0.0;
      }
    for (int j = -1; j < nj; ++j)
      for (int i = 0; i < ni; ++i) {
        double fbar = kappa ? -(MU(i, j) - MU(i, j + 1)) : -coeff * (LAM(i, j) - LAM(i, j + 1));
        gy[(size_t)(j + 1) * (size_t)ni + (size_t)i] = my[MYIDX(i, j, k)] ? fbar : 0.0;
      }
    /* lap(q) enters Fx(q-ei) with +1 and Fx(q) with -1 (same for y). */
    for (int j = -1; j <= nj; ++j)
      for (int i = -1; i <= ni; ++i)
        lb[(size_t)(j + 1) * (size_t)li + (size_t)(i + 1)] =
            (GX(i - 1, j) - GX(i, j)) + (GY(i, j - 1) - GY(i, j));
    /* stated form: lap(q) = 4u(q) - u(q+-ei) - u(q+-ej); the damping form
     * is its negative.  Plus the identity term of out. */
    for (int j = -2; j < nj + 2; ++j)
      for (int i = -2; i < ni + 2; ++i) {
        double nb = LB(i + 1, j) + LB(i - 1, j) + LB(i, j + 1) + LB(i, j - 1);
        double v = damping ? LAM(i, j) + (nb - 4.0 * LB(i, j))
                           : LAM(i, j) + 4.0 * LB(i, j) - LB(i + 1, j) - LB(i - 1, j) -
                                 LB(i, j + 1) - LB(i, j - 1);
        ubar[UIDX(i, j, k)] = v;
      }
  }
#undef INI
#undef LAM
#undef MU
#undef GX
#undef GY
#undef LB
  free(gx);
  free(gy);
  free(lb);
  }
}

void oracle_hdiff_adjoint(int ni, int nj, int nk, const double* lam, const unsigned char* mx,
                          const unsigned char* my, double coeff, double* ubar) {
  oracle_hdiff_adjoint_gen(ni, nj, nk, lam, mx, my, coeff, NULL, 0, ubar);
}

/* Vertical advection adjoint: lam = T^{-T} xbar.  T^T has sub-diagonal
 * c_{k-1}, diagonal b_k and super-diagonal a_{k+1}; solved by a fresh
 * Thomas elimination on that transposed matrix. */
void oracle_vadv_adjoint(int ni, int nj, int nk, const double* xbar, const double* w, double dt_dz,
                         double* lam) {
  if (ni <= 0 || nj <= 0 || nk <= 0) return;
#pragma omp parallel
  { /* columns are independent: one pair of column temporaries per thread */
  double* al = (double*)malloc(sizeof(double) * (size_t)nk);
  double* be = (double*)malloc(sizeof(double) * (size_t)nk);
#pragma omp for schedule(static)
  for (int j = 0; j < nj; ++j)
    for (int i = 0; i < ni; ++i) {
      for (int k = 0; k < nk; ++k) {
        double sub = k >= 1 ? coef_c(w, ni, nj, nk, i, j, k - 1, dt_dz) : 0.0;
        double sup = k <= nk - 2 ? coef_a(w, ni, nj, i, j, k + 1, dt_dz) : 0.0;
        double ak = coef_a(w, ni, nj, i, j, k, dt_dz);
        double ck = coef_c(w, ni, nj, nk, i, j, k, dt_dz);
        double diag = 1.0 + fabs(ak) + fabs(ck);
        double rhs = xbar[IIDX(i, j, k)];
        if (k == 0) {
          al[0] = sup / diag;
          be[0] = rhs / diag;
        } else {
          double m = diag - sub * al[k - 1];
          al[k] = sup / m;
          be[k] = (rhs - sub * be[k - 1]) / m;
        }
      }
      lam[IIDX(i, j, nk - 1)] = be[nk - 1];
      for (int k = nk - 2; k >= 0; --k) lam[IIDX(i, j, k)] = be[k] - al[k] * lam[IIDX(i, j, k + 1)];
    }
  free(al);
  free(be);
  }
}

/* Step adjoint: lam = T^{-T} xbar; ubar = J_h^T lam; databar = lam. */
void oracle_step_adjoint_gen(int ni, int nj, int nk, const double* xbar, const double* w,
                             const unsigned char* mx, const unsigned char* my, double coeff,
                             const double* kappa, int damping, double dt_dz, double* ubar,
                             double* databar) {
  size_t n = (size_t)ni * (size_t)nj * (size_t)nk;
  double* lam = (double*)malloc(sizeof(double) * (n > 0 ? n : 1));
  oracle_vadv_adjoint(ni, nj, nk, xbar, w, dt_dz, lam);
  oracle_hdiff_adjoint_gen(ni, nj, nk, lam, mx, my, coeff, kappa, damping, ubar);
  if (databar) memcpy(databar, lam, sizeof(double) * n);
  free(lam);
}

void oracle_step_adjoint(int ni, int nj, int nk, const double* xbar, const double* w,
                         const unsigned char* mx, const unsigned char* my, double coeff,
                         double dt_dz, double* ubar, double* databar) {
  oracle_step_adjoint_gen(ni, nj, nk, xbar, w, mx, my, coeff, NULL, 0, dt_dz, ubar, databar);
}

/* Tangent-linear step with masks held fixed: dx = T^{-1} (J_h v). `v` is
 * padded, `dx` interior.  No forcing term (data enters additively). */
void oracle_step_tangent_gen(int ni, int nj, int nk, const double* v, const double* w,
                             const unsigned char* mx, const unsigned char* my, double coeff,
                             const double* kappa, int damping, double dt_dz, double* dx) {
  size_t n = (size_t)ni * (size_t)nj * (size_t)nk;
  if (n == 0) return;
  double* h = (double*)malloc(sizeof(double) * n);
  hdiff_with_masks(ni, nj, nk, v, coeff, kappa, damping, mx, my, h);
  thomas_columns(ni, nj, nk, h, w, dt_dz, dx);
  free(h);
}

void oracle_step_tangent(int ni, int nj, int nk, const double* v, const double* w,
                         const unsigned char* mx, const unsigned char* my, double coeff,
                         double dt_dz, double* dx) {
  oracle_step_tangent_gen(ni, nj, nk, v, w, mx, my, coeff, NULL, 0, dt_dz, dx);
}

/* Tangent of the horizontal diffusion alone (interior output). */
void oracle_hdiff_tangent_gen(int ni, int nj, int nk, const double* v, const unsigned char* mx,
                              const unsigned char* my, double coeff, const double* kappa,
                              int damping, double* dh) {
  if ((size_t)ni * (size_t)nj * (size_t)nk == 0) return;
  hdiff_with_masks(ni, nj, nk, v, coeff, kappa, damping, mx, my, dh);
}

void oracle_hdiff_tangent(int ni, int nj, int nk, const double* v, const unsigned char* mx,
                          const unsigned char* my, double coeff, double* dh) {
  oracle_hdiff_tangent_gen(ni, nj, nk, v, mx, my, coeff, NULL, 0, dh);
}

/* Tridiagonal matrix-vector product y = T x per column (for residual pins). */
void oracle_tridiag_apply(int ni, int nj, int nk, const double* x, const double* w, double dt_dz,
                          double* y) {
  for (int j = 0; j < nj; ++j)
    for (int i = 0; i < ni; ++i)
      for (int k = 0; k < nk; ++k) {
        double a = coef_a(w, ni, nj, i, j, k, dt_dz);
        double c = coef_c(w, ni, nj, nk, i, j, k, dt_dz);
        double b = 1.0 + fabs(a) + fabs(c);
        double v = b * x[IIDX(i, j, k)];
        if (k >= 1) v += a * x[IIDX(i, j, k - 1)];
        if (k <= nk - 2) v += c * x[IIDX(i, j, k + 1)];
        y[IIDX(i, j, k)] = v;
      }
}

/* The Laplacian stage alone on the box [-1, ni] x [-1, nj]:
 * lap[k][j+1][i+1], shape [nk][nj+2][ni+2]. */
void oracle_laplacian(int ni, int nj, int nk, const double* u, double* lap) {
  for (int k = 0; k < nk; ++k)
    for (int j = -1; j <= nj; ++j)
      for (int i = -1; i <= ni; ++i)
        lap[(size_t)k * (size_t)(nj + 2) * (size_t)(ni + 2) + (size_t)(j + 1) * (size_t)(ni + 2) +
            (size_t)(i + 1)] = lap64(u, ni, nj, i, j, k, 0);
}

/* ------------------------------------------------------------------ */
/* Periodic boundaries: the 2-point halo of a padded field holds the     */
/* interior values at the wrapped indices (i mod ni, j mod nj), corners  */
/* included.  In place on a padded [nk][nj+4][ni+4] array.              */
/* ------------------------------------------------------------------ */
static int wrap(int i, int n) { int r = i % n; return r < 0 ? r + n : r; }

void oracle_halo_periodic(int ni, int nj, int nk, double* u) {
  if (ni <= 0 || nj <= 0) return;
  for (int k = 0; k < nk; ++k)
    for (int j = -2; j < nj + 2; ++j)
      for (int i = -2; i < ni + 2; ++i) {
        if (i >= 0 && i < ni && j >= 0 && j < nj) continue;
        u[UIDX(i, j, k)] = u[UIDX(wrap(i, ni), wrap(j, nj), k)];
      }
}

/* ------------------------------------------------------------------ */
/* Parameter gradients of one step (parameter tuning).                  */
/* With the limiter decisions held fixed the diffusion is               */
/*   h = u - coeff * D(u),  D(u)(p) = (Fx(p) - Fx(p-ei)) + (Fy(p) - Fy(p-ej)) */
/* (the limited fluxes do not depend on coeff), and the column solve is */
/* T(w) x = h + data.  For a scalar loss L with xbar = dL/dx and        */
/* lam = T^{-T} xbar:                                                   */
/*   dL/dcoeff = sum_p lam(p) dh(p)/dcoeff = -sum_p lam(p) D(u)(p),      */
/*   dL/dT(k,l) = -lam_k x_l for every nonzero entry of T: a_k (l=k-1), */
/*   b_k (l=k), c_k (l=k+1), chained through the coefficient            */
/*   definitions a_k = -r/4 w_k, c_k = r/4 w_{k+1}, b_k = 1+|a_k|+|c_k| */
/*   (d|t|/dt = sign t, taken as 0 at t = 0).                           */
/* ------------------------------------------------------------------ */

/* D(u) on the interior with the given masks (interior layout), for the
 * Laplacian of the given form. */
void oracle_hdiff_divergence_form(int ni, int nj, int nk, const double* u, const unsigned char* mx,
                                  const unsigned char* my, int damping, double* div) {
  if ((size_t)ni * (size_t)nj * (size_t)nk == 0) return;
  /* h = u - 1 * D would round; take the flux differences directly */
  const int li = ni + 2, lj = nj + 2;
  double* lap = (double*)malloc(sizeof(double) * (size_t)li * (size_t)lj);
#define LAPD(i, j) lap[(size_t)((j) + 1) * (size_t)li + (size_t)((i) + 1)]
  for (int k = 0; k < nk; ++k) {
    for (int j = -1; j <= nj; ++j)
      for (int i = -1; i <= ni; ++i) LAPD(i, j) = lap64(u, ni, nj, i, j, k, damping);
    for (int j = 0; j < nj; ++j)
      for (int i = 0; i < ni; ++i) {
        double fxr = mx[MXIDX(i, j, k)] ? LAPD(i + 1, j) - LAPD(i, j) : 0.0;
        double fxl = mx[MXIDX(i - 1, j, k)] ? LAPD(i, j) - LAPD(i - 1, j) : 0.0;
        double fyr = my[MYIDX(i, j, k)] ? LAPD(i, j + 1) - LAPD(i, j) : 0.0;
        double fyl = my[MYIDX(i, j - 1, k)] ? LAPD(i, j) - LAPD(i, j - 1) : 0.0;
        div[IIDX(i, j, k)] = (fxr - fxl) + (fyr - fyl);
      }
  }
#undef LAPD
  free(lap);
}

void oracle_hdiff_divergence(int ni, int nj, int nk, const double* u, const unsigned char* mx,
                             const unsigned char* my, double* div) {
  oracle_hdiff_divergence_form(ni, nj, nk, u, mx, my, 0, div);
}

/* dL/dcoeff = -sum lam * D(u), D with the masks and Laplacian form given;
 * the sum is compensated (Neumaier) so that it is accurate to about one
 * rounding. */
double oracle_coeff_grad_form(int ni, int nj, int nk, const double* u, const double* lam,
                              const unsigned char* mx, const unsigned char* my, int damping) {
  size_t n = (size_t)ni * (size_t)nj * (size_t)nk;
  if (n == 0) return 0.0;
  double* div = (double*)malloc(sizeof(double) * n);
  oracle_hdiff_divergence_form(ni, nj, nk, u, mx, my, damping, div);
  double s = 0.0, comp = 0.0;
  for (size_t p = 0; p < n; ++p) {
    double t = -(lam[p] * div[p]);
    double v = s + t;
    comp += fabs(s) >= fabs(t) ? (s - v) + t : (t - v) + s;
    s = v;
  }
  free(div);
  return s + comp;
}

double oracle_coeff_grad(int ni, int nj, int nk, const double* u, const double* lam,
                         const unsigned char* mx, const unsigned char* my) {
  return oracle_coeff_grad_form(ni, nj, nk, u, lam, mx, my, 0);
}

/* Gradient with respect to a per-point coefficient field: out(p) depends on
 * kappa(p) alone, through -kappa(p) D(u)(p), so dL/dkappa(p) = -lam(p) D(u)(p)
 * (interior layout). */
void oracle_coeff_field_grad(int ni, int nj, int nk, const double* u, const double* lam,
                             const unsigned char* mx, const unsigned char* my, int damping,
                             double* kbar) {
  size_t n = (size_t)ni * (size_t)nj * (size_t)nk;
  if (n == 0) return;
  oracle_hdiff_divergence_form(ni, nj, nk, u, mx, my, damping, kbar);
  for (size_t p = 0; p < n; ++p) kbar[p] = -(lam[p] * kbar[p]);
}

static double sgn(double t) { return t > 0.0 ? 1.0 : (t < 0.0 ? -1.0 : 0.0); }

/* dL/dw on the staggered levels 0..nk (w_0 and w_nk do not enter T, so
 * their gradient is 0); lam and x interior, wbar staggered. */
void oracle_w_grad(int ni, int nj, int nk, const double* w, const double* x, const double* lam,
                   double dt_dz, double* wbar) {
  const size_t plane = (size_t)ni * (size_t)nj;
  for (size_t p = 0; p < plane * (size_t)(nk + 1); ++p) wbar[p] = 0.0;
  const double q = 0.25 * dt_dz;
  for (int j = 0; j < nj; ++j)
    for (int i = 0; i < ni; ++i)
      for (int k = 0; k < nk; ++k) {
        const double lk = lam[IIDX(i, j, k)];
        const double a = coef_a(w, ni, nj, i, j, k, dt_dz);
        const double c = coef_c(w, ni, nj, nk, i, j, k, dt_dz);
        const double bbar = -lk * x[IIDX(i, j, k)];
        if (k >= 1) { /* a_k = -q w_k, |a_k| in b_k */
          const double abar = -lk * x[IIDX(i, j, k - 1)];
          wbar[(size_t)k * plane + (size_t)j * (size_t)ni + (size_t)i] += -q * abar + sgn(a) * (-q) * bbar;
        }
        if (k <= nk - 2) { /* c_k = q w_{k+1}, |c_k| in b_k */
          const double cbar = -lk * x[IIDX(i, j, k + 1)];
          wbar[(size_t)(k + 1) * plane + (size_t)j * (size_t)ni + (size_t)i] += q * cbar + sgn(c) * q * bbar;
        }
      }
}

int oracle_version(void) { return 2; }

/* Threads a parallel region of this build uses: 1 unless built with OpenMP. */
int oracle_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
