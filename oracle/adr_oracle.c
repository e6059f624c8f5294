/*
 * CPU oracle for the ILU(0)-preconditioned BiCGSTAB solver of the 2-D steady
 * advection-diffusion problem of Datta & Carrasco Heres, "Numerical Solution of
 * Advection-Diffusion Equation Using Preconditioner as Incomplete LU
 * Decomposition and the BiCGSTAB Acceleration Method" (arXiv:1308.5215).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, sequential FP64
 * statement of what the GPU library computes.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * source with the GPU library and includes nothing from it.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -shared -fPIC
 * (contraction is off so that every fused multiply-add below is the explicit
 * fma() that is written, and nothing else is fused).
 *
 * Index convention: interior unknown (i, j), 0 <= i < nx, 0 <= j < ny, is
 * stored at k = j*nx + i (x fastest), the lexicographic ordering of the
 * paper's assembly routine (appendix, Matrix_A_b_U).  Interior node (i, j)
 * sits at x = (i+1)*dx, y = (j+1)*dy with dx = X/(nx+1), dy = Y/(ny+1), i.e.
 * nx = m-1, ny = n-1 for the paper's m, n intervals.
 *
 * Every function cites the passage of the paper it follows.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Status codes (same numbering as the library's public header; written out
 * here again on purpose: the oracle includes nothing from the library). */
enum {
  OR_OK = 0,
  OR_ERR_ARG = -1,
  OR_MAXIT = 1,
  OR_BREAKDOWN_RHO = 2,
  OR_OMEGA_ZERO = 3,
  OR_ZERO_PIVOT = 4,
  OR_NONFINITE = 5,
  OR_INACCURATE = 6
};

/* ------------------------------------------------------------------------ */
/* Section 2-3: problem data.                                               */
/* ------------------------------------------------------------------------ */

/* Manufactured solution of Section 2: u = exp(-x/X) (1 - exp(-y/Y)) y. */
double or_u_exact(double x, double y, double X, double Y) {
  return (exp(-x / X) * (1.0 - exp(-y / Y))) * y;
}

/* 1-D tables of the discretisation (Section 4 and the assembly routine of the
 * appendix): node coordinates by multiplication (not accumulation),
 * a_i = 1 + x_i^2, b_j = X exp(-y_j), and the three exponentials the
 * manufactured forcing of Section 3 is built from.  Any output may be NULL. */
void or_tables(double X, double Y, int32_t nx, int32_t ny,
               double *x, double *y, double *a, double *b,
               double *ex, double *ey, double *eb) {
  const double dx = X / (double)(nx + 1), dy = Y / (double)(ny + 1);
  for (int32_t i = 0; i < nx; ++i) {
    const double xi = (double)(i + 1) * dx;
    if (x) x[i] = xi;
    if (a) a[i] = 1.0 + xi * xi;
    if (ex) ex[i] = exp(-xi / X);
  }
  for (int32_t j = 0; j < ny; ++j) {
    const double yj = (double)(j + 1) * dy;
    if (y) y[j] = yj;
    if (eb) eb[j] = exp(-yj);
    if (b) b[j] = X * exp(-yj);
    if (ey) ey[j] = exp(-yj / Y);
  }
}

/* Manufactured forcing f = eps*(u_xx + u_yy) + a u_x + b u_y of Section 3, in
 * the three-term form T1 + T2 + T3 of the appendix's main driver (the printed
 * formula in Section 3 is garbled; the derivatives it starts from agree with
 * this form).  The exponential of a sum is taken as the product of the 1-D
 * exponentials: exp(-(x/X + y/Y)) = exp(-x/X) exp(-y/Y).  Evaluation order is
 * left to right as written, with no contraction. */
double or_f_point(double eps, double X, double Y, double x, double y,
                  double a, double ex, double ey, double eb) {
  const double X2 = X * X, Y2 = Y * Y;
  const double exy = ex * ey;
  const double t1 = eps * ((y / X2) * ex + ((2.0 / Y - y / Y2) - y / X2) * exy);
  const double ya = (y * a) / X;
  const double t2 = ex * (X * eb - ya);
  const double t3 = exy * ((ya - X * eb) + ((X / Y) * y) * eb);
  return (t1 + t2) + t3;
}

/* Boundary data: Dirichlet values u(0,y_j), u(X,y_j), u(x_i,0), u(x_i,Y) and
 * the Neumann data g_x(y_j) = du/dx(X,y_j), g_y(x_i) = du/dy(x_i,Y) of
 * Section 2, evaluated from the manufactured u as the appendix drivers do.
 * Arrays of length ny (x-edges) and nx (y-edges); any output may be NULL. */
void or_boundary(double X, double Y, int32_t nx, int32_t ny,
                 double *u_x0, double *u_xX, double *u_y0, double *u_yY,
                 double *g_xX, double *g_yY) {
  const double dx = X / (double)(nx + 1), dy = Y / (double)(ny + 1);
  const double e1 = exp(-1.0);
  for (int32_t j = 0; j < ny; ++j) {
    const double yj = (double)(j + 1) * dy;
    const double ey = exp(-yj / Y);
    if (u_x0) u_x0[j] = (1.0 - ey) * yj;
    if (u_xX) u_xX[j] = (e1 * (1.0 - ey)) * yj;
    if (g_xX) g_xX[j] = (((-1.0 / X) * e1) * (1.0 - ey)) * yj;
  }
  for (int32_t i = 0; i < nx; ++i) {
    const double xi = (double)(i + 1) * dx;
    const double ex = exp(-xi / X);
    if (u_y0) u_y0[i] = 0.0;
    if (u_yY) u_yY[i] = (ex * (1.0 - e1)) * Y;
    /* du/dy at y = Y: exp(-x/X) [ (Y/Y) exp(-Y/Y) + (1 - exp(-Y/Y)) ] */
    if (g_yY) g_yY[i] = ex * (e1 + (1.0 - e1));
  }
}

/* Manufactured forcing on every interior node (N = nx*ny values). */
void or_forcing(double eps, double X, double Y, int32_t nx, int32_t ny, double *f) {
  double *x = malloc(sizeof(double) * (size_t)nx), *a = malloc(sizeof(double) * (size_t)nx);
  double *ex = malloc(sizeof(double) * (size_t)nx);
  double *y = malloc(sizeof(double) * (size_t)ny), *ey = malloc(sizeof(double) * (size_t)ny);
  double *eb = malloc(sizeof(double) * (size_t)ny);
  or_tables(X, Y, nx, ny, x, y, a, NULL, ex, ey, eb);
  for (int32_t j = 0; j < ny; ++j)
    for (int32_t i = 0; i < nx; ++i)
      f[(size_t)j * nx + i] = or_f_point(eps, X, Y, x[i], y[j], a[i], ex[i], ey[j], eb[j]);
  free(x); free(a); free(ex); free(y); free(ey); free(eb);
}

/* ------------------------------------------------------------------------ */
/* Section 4: assembly into five diagonals.                                 */
/* ------------------------------------------------------------------------ */

/* Five-point matrix and right-hand side, Section 4, every equation
 * multiplied by dx^2 dy^2.
 *   upwind ("hybrid") scheme: second differences centred, first differences
 *   backward:  S = eps dx^2 - b dx^2 dy,  W = eps dy^2 - a dx dy^2,
 *              C = -2 eps dy^2 - 2 eps dx^2 + a dx dy^2 + b dx^2 dy,
 *              E = eps dy^2,             N = eps dx^2;
 *   centered scheme:  S = eps dx^2 - b dx^2 dy / 2,  W = eps dy^2 - a dx dy^2 / 2,
 *              C = -2 eps dy^2 - 2 eps dx^2,
 *              E = eps dy^2 + a dx dy^2 / 2,  N = eps dx^2 + b dx^2 dy / 2.
 * rhs = f dx^2 dy^2, minus the couplings to boundary nodes times the boundary
 * values (the appendix's order: y = 0, y = Y, x = 0, x = X).
 * bc = 1 (Neumann on x = X and y = Y): the boundary node is eliminated by the
 * one-sided difference U_boundary = U_interior + h g (Neumann assembly routines
 * of the appendix), i.e. C += E (resp. N) and rhs -= E dx g_x (resp. N dy g_y);
 * on the corner node the x-edge term is added first.
 * Couplings to boundary nodes are stored as 0.
 * Problem data, as the appendix's assembly routines take it (each NULL for
 * the manufactured problem of Sections 2-3):
 *   f_user  forcing at every interior node (nx*ny values);
 *   u_x0    u(0, y_j) (ny values);  u_xX  u(X, y_j), or g_x(y_j) = du/dx for bc = 1;
 *   u_y0    u(x_i, 0) (nx values);  u_yY  u(x_i, Y), or g_y(x_i) = du/dy for bc = 1.
 * forcing: NULL, or a perturbation added to the manufactured f:
 * f = f_man + amp * max|f_man| * g with g = forcing (nx*ny values), the max
 * taken over interior nodes (ignored when f_user is given).
 * Returns OR_OK or OR_ERR_ARG. */
int or_assemble_data(double eps, double X, double Y, int32_t nx, int32_t ny,
                     int32_t scheme, int32_t bc, const double *f_user,
                     const double *forcing, double amp,
                     const double *u_x0_user, const double *u_xX_user,
                     const double *u_y0_user, const double *u_yY_user,
                     double *S, double *W, double *C, double *E, double *N, double *rhs) {
  if (!(eps > 0.0) || !(X > 0.0) || !(Y > 0.0) || nx < 1 || ny < 1 ||
      (scheme != 0 && scheme != 1) || (bc != 0 && bc != 1))
    return OR_ERR_ARG;
  const size_t n = (size_t)nx * (size_t)ny;
  const double dx = X / (double)(nx + 1), dy = Y / (double)(ny + 1);
  const double dx2 = dx * dx, dy2 = dy * dy;
  const double cx = eps * dy2;      /* diffusion weight of x-neighbours */
  const double cy = eps * dx2;      /* diffusion weight of y-neighbours */
  const double gx = dx * dy2;       /* weight of a u_x term */
  const double gy = dx2 * dy;       /* weight of a u_y term */
  const double scale = dx2 * dy2;
  double *x = malloc(sizeof(double) * (size_t)nx), *a = malloc(sizeof(double) * (size_t)nx);
  double *ex = malloc(sizeof(double) * (size_t)nx);
  double *y = malloc(sizeof(double) * (size_t)ny), *b = malloc(sizeof(double) * (size_t)ny);
  double *ey = malloc(sizeof(double) * (size_t)ny), *eb = malloc(sizeof(double) * (size_t)ny);
  double *u_x0 = malloc(sizeof(double) * (size_t)ny), *u_xX = malloc(sizeof(double) * (size_t)ny);
  double *g_xX = malloc(sizeof(double) * (size_t)ny);
  double *u_y0 = malloc(sizeof(double) * (size_t)nx), *u_yY = malloc(sizeof(double) * (size_t)nx);
  double *g_yY = malloc(sizeof(double) * (size_t)nx);
  or_tables(X, Y, nx, ny, x, y, a, b, ex, ey, eb);
  or_boundary(X, Y, nx, ny, u_x0, u_xX, u_y0, u_yY, g_xX, g_yY);

  /* user boundary data replaces the manufactured values */
  if (u_x0_user) memcpy(u_x0, u_x0_user, sizeof(double) * (size_t)ny);
  if (u_xX_user) memcpy(bc == 0 ? u_xX : g_xX, u_xX_user, sizeof(double) * (size_t)ny);
  if (u_y0_user) memcpy(u_y0, u_y0_user, sizeof(double) * (size_t)nx);
  if (u_yY_user) memcpy(bc == 0 ? u_yY : g_yY, u_yY_user, sizeof(double) * (size_t)nx);

  /* forcing */
  if (f_user) {
    memcpy(rhs, f_user, sizeof(double) * n);
    forcing = NULL;
  } else {
    for (int32_t j = 0; j < ny; ++j)
      for (int32_t i = 0; i < nx; ++i)
        rhs[(size_t)j * nx + i] = or_f_point(eps, X, Y, x[i], y[j], a[i], ex[i], ey[j], eb[j]);
  }
  if (forcing) {
    double fmax = 0.0;
    for (size_t k = 0; k < n; ++k) {
      const double v = fabs(rhs[k]);
      if (v > fmax) fmax = v;
    }
    const double c = amp * fmax;
    for (size_t k = 0; k < n; ++k) rhs[k] = rhs[k] + c * forcing[k];
  }

  for (int32_t j = 0; j < ny; ++j) {
    for (int32_t i = 0; i < nx; ++i) {
      const size_t k = (size_t)j * nx + i;
      double s, w, c, e, nn;
      if (scheme == 0) {
        w = cx - a[i] * gx;
        e = cx;
        s = cy - b[j] * gy;
        nn = cy;
        c = (a[i] * gx + b[j] * gy) - 2.0 * (cx + cy);
      } else {
        w = cx - 0.5 * (a[i] * gx);
        e = cx + 0.5 * (a[i] * gx);
        s = cy - 0.5 * (b[j] * gy);
        nn = cy + 0.5 * (b[j] * gy);
        c = -2.0 * (cx + cy);
      }
      double r = scale * rhs[k];
      /* boundary lifting, appendix order: y = 0, y = Y, x = 0, x = X */
      if (j == 0) r = r - s * u_y0[i];
      if (j == ny - 1) {
        if (bc == 0) r = r - nn * u_yY[i];
        else r = r - (nn * dy) * g_yY[i];
      }
      if (i == 0) r = r - w * u_x0[j];
      if (i == nx - 1) {
        if (bc == 0) r = r - e * u_xX[j];
        else r = r - (e * dx) * g_xX[j];
      }
      if (bc == 1) {
        if (i == nx - 1) c = c + e;
        if (j == ny - 1) c = c + nn;
      }
      S[k] = (j == 0) ? 0.0 : s;
      W[k] = (i == 0) ? 0.0 : w;
      C[k] = c;
      E[k] = (i == nx - 1) ? 0.0 : e;
      N[k] = (j == ny - 1) ? 0.0 : nn;
      rhs[k] = r;
    }
  }
  free(x); free(a); free(ex); free(y); free(b); free(ey); free(eb);
  free(u_x0); free(u_xX); free(g_xX); free(u_y0); free(u_yY); free(g_yY);
  return OR_OK;
}

/* The manufactured problem, optionally with a forcing perturbation (see
 * or_assemble_data). */
int or_assemble(double eps, double X, double Y, int32_t nx, int32_t ny,
                int32_t scheme, int32_t bc, const double *forcing, double amp,
                double *S, double *W, double *C, double *E, double *N, double *rhs) {
  return or_assemble_data(eps, X, Y, nx, ny, scheme, bc, NULL, forcing, amp, NULL, NULL, NULL, NULL,
                          S, W, C, E, N, rhs);
}

/* ------------------------------------------------------------------------ */
/* Instance classification (Section 6.3, mesh Reynolds number).             */
/* ------------------------------------------------------------------------ */

/* What the discretisation of one instance looks like before it is solved.
 *   pe_x, pe_y  cell Peclet (mesh Reynolds) numbers max_i a_i dx / eps and
 *               max_j b_j dy / eps over the interior nodes (Section 6.3: the
 *               centered scheme stays free of oscillations below 2);
 *   g_y         X (1 - exp(-Y)) / eps, the integral of b(y)/eps over [0, Y]:
 *               with Neumann data on x = X, y = Y the closed operator grows
 *               like exp(g_y) (the paper observes that low eps makes the
 *               Neumann condition fail, Section 6.1);
 *   neg_offdiag couplings S, W, E, N between interior unknowns that are < 0
 *               (none: -A has the sign pattern of an M-matrix);
 *   nonneg_diag interior points with C >= 0 (the diagonal changes sign, and
 *               the ILU(0) pivots can pass through zero);
 *   expect_fail 1 if the solve is expected not to reach ||b - A x|| < tol ||b||:
 *               - Neumann data with g_y > ln(tol / u), u = 2^-53: the true
 *                 residual cannot fall below about u exp(g_y);
 *               - a diagonal that changes sign inside the grid
 *                 (0 < nonneg_diag < N);
 *               - the upwind ("hybrid") scheme, whose backward differences
 *                 are downwind for eq. (1), with a negative diagonal and a
 *                 cell Peclet number above 2 (the Section 6.3 threshold).
 * Computed from the assembled five diagonals, point by point. */
typedef struct {
  double pe_x, pe_y, g_y;
  int64_t neg_offdiag, nonneg_diag;
  int32_t expect_fail, pad;
} or_class;

int or_classify(double eps, double X, double Y, int32_t nx, int32_t ny, int32_t scheme, int32_t bc,
                double tol, or_class *out) {
  memset(out, 0, sizeof(*out));
  if (!(eps > 0.0) || !(X > 0.0) || !(Y > 0.0) || nx < 1 || ny < 1 ||
      (scheme != 0 && scheme != 1) || (bc != 0 && bc != 1))
    return OR_ERR_ARG;
  const size_t n = (size_t)nx * (size_t)ny;
  double *S = malloc(sizeof(double) * n), *W = malloc(sizeof(double) * n), *C = malloc(sizeof(double) * n);
  double *E = malloc(sizeof(double) * n), *N = malloc(sizeof(double) * n), *r = malloc(sizeof(double) * n);
  or_assemble(eps, X, Y, nx, ny, scheme, bc, NULL, 0.0, S, W, C, E, N, r);
  const double dx = X / (double)(nx + 1), dy = Y / (double)(ny + 1);
  double amax = 0.0, bmax = 0.0;
  for (int32_t i = 0; i < nx; ++i) {
    const double xi = (double)(i + 1) * dx;
    const double a = 1.0 + xi * xi;
    if (a > amax) amax = a;
  }
  for (int32_t j = 0; j < ny; ++j) {
    const double b = X * exp(-(double)(j + 1) * dy);
    if (b > bmax) bmax = b;
  }
  out->pe_x = amax * dx / eps;
  out->pe_y = bmax * dy / eps;
  out->g_y = X * (1.0 - exp(-Y)) / eps;
  for (size_t k = 0; k < n; ++k) {
    out->neg_offdiag += (S[k] < 0.0) + (W[k] < 0.0) + (E[k] < 0.0) + (N[k] < 0.0);
    out->nonneg_diag += (C[k] >= 0.0);
  }
  const double pe = out->pe_x > out->pe_y ? out->pe_x : out->pe_y;
  const int neumann_floor = bc == 1 && tol > 0.0 && out->g_y > log(tol / ldexp(1.0, -53));
  const int sign_change = out->nonneg_diag > 0 && out->nonneg_diag < (int64_t)n;
  const int downwind = scheme == 0 && out->nonneg_diag == 0 && pe > 2.0;
  out->expect_fail = neumann_floor || sign_change || downwind;
  free(S); free(W); free(C); free(E); free(N); free(r);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Five-point operator.                                                     */
/* ------------------------------------------------------------------------ */

/* v = A x for the five-diagonal A; neighbours outside the grid contribute 0.
 * Fixed evaluation: fma(N,x_n, fma(E,x_e, fma(W,x_w, fma(S,x_s, C*x_c)))). */
void or_spmv(int32_t nx, int32_t ny, const double *S, const double *W, const double *C,
             const double *E, const double *N, const double *x, double *v) {
  for (int32_t j = 0; j < ny; ++j)
    for (int32_t i = 0; i < nx; ++i) {
      const size_t k = (size_t)j * nx + i;
      const double xs = (j > 0) ? x[k - nx] : 0.0;
      const double xw = (i > 0) ? x[k - 1] : 0.0;
      const double xe = (i < nx - 1) ? x[k + 1] : 0.0;
      const double xn = (j < ny - 1) ? x[k + nx] : 0.0;
      double t = C[k] * x[k];
      t = fma(S[k], xs, t);
      t = fma(W[k], xw, t);
      t = fma(E[k], xe, t);
      t = fma(N[k], xn, t);
      v[k] = t;
    }
}

/* ------------------------------------------------------------------------ */
/* Section 5.1: ILU(0) (Saad), the no-fill incomplete factorisation whose     */
/* pattern is that of A.                                                     */
/* ------------------------------------------------------------------------ */

/* For the five-point matrix, ILU(0) keeps L unit lower with entries at
 * (k,k-1) and (k,k-nx), and U with the diagonal d and A's own upper entries
 * E (k,k+1) and N (k,k+nx).  Elimination in natural order drops the fill at
 * (k,k-nx+1) and (k,k+nx-1), which leaves the pivot recurrence
 *   lw_k = W_k / d_{k-1},  ls_k = S_k / d_{k-nx},
 *   d_k  = C_k - lw_k E_{k-1} - ls_k N_{k-nx}.
 * Stored: invd = 1/d (correctly rounded division), lw = W*invd_{k-1},
 * ls = S*invd_{k-nx}; d = fma(-ls, N_{k-nx}, fma(-lw, E_{k-1}, C)).
 * Returns OR_ZERO_PIVOT (with *bad = k) at the first zero or non-finite
 * pivot, OR_OK otherwise. */
int or_ilu0(int32_t nx, int32_t ny, const double *S, const double *W, const double *C,
            const double *E, const double *N, double *lw, double *ls, double *invd,
            int64_t *bad) {
  const size_t n = (size_t)nx * (size_t)ny;
  for (size_t k = 0; k < n; ++k) {
    const int32_t i = (int32_t)(k % (size_t)nx);
    const int32_t j = (int32_t)(k / (size_t)nx);
    const double lwk = (i > 0) ? W[k] * invd[k - 1] : 0.0;
    const double lsk = (j > 0) ? S[k] * invd[k - nx] : 0.0;
    const double ew = (i > 0) ? E[k - 1] : 0.0;
    const double ns = (j > 0) ? N[k - nx] : 0.0;
    double d = fma(-lwk, ew, C[k]);
    d = fma(-lsk, ns, d);
    lw[k] = lwk;
    ls[k] = lsk;
    if (d == 0.0 || !isfinite(d)) {
      if (bad) *bad = (int64_t)k;
      invd[k] = 0.0;
      return OR_ZERO_PIVOT;
    }
    invd[k] = 1.0 / d;
  }
  if (bad) *bad = -1;
  return OR_OK;
}

/* Forward substitution with the unit lower factor: y = L^{-1} q,
 *   y_k = q_k - lw_k y_{k-1} - ls_k y_{k-nx}  = fma(-ls, y_s, fma(-lw, y_w, q)). */
void or_lsolve(int32_t nx, int32_t ny, const double *lw, const double *ls,
               const double *q, double *y) {
  const size_t n = (size_t)nx * (size_t)ny;
  for (size_t k = 0; k < n; ++k) {
    const int32_t i = (int32_t)(k % (size_t)nx);
    const int32_t j = (int32_t)(k / (size_t)nx);
    const double yw = (i > 0) ? y[k - 1] : 0.0;
    const double ys = (j > 0) ? y[k - nx] : 0.0;
    double t = fma(-lw[k], yw, q[k]);
    t = fma(-ls[k], ys, t);
    y[k] = t;
  }
}

/* Backward substitution with the upper factor U = diag(d) + (ue at k+1,
 * un at k+nx): z = U^{-1} y,
 *   z_k = (y_k - ue_k z_{k+1} - un_k z_{k+nx}) / d_k
 *       = fma(-un, z_n, fma(-ue, z_e, y)) * invd.
 * For ILU(0), ue = E and un = N of A. */
void or_usolve(int32_t nx, int32_t ny, const double *ue, const double *un,
               const double *invd, const double *y, double *z) {
  const size_t n = (size_t)nx * (size_t)ny;
  for (size_t kk = n; kk-- > 0;) {
    const int32_t i = (int32_t)(kk % (size_t)nx);
    const int32_t j = (int32_t)(kk / (size_t)nx);
    const double ze = (i < nx - 1) ? z[kk + 1] : 0.0;
    const double zn = (j < ny - 1) ? z[kk + nx] : 0.0;
    double t = fma(-ue[kk], ze, y[kk]);
    t = fma(-un[kk], zn, t);
    z[kk] = t * invd[kk];
  }
}

/* The same two substitutions carried out in single precision (the mixed-
 * precision preconditioner in which the factors are stored in FP32 and the
 * triangular solves themselves run in FP32): inputs are rounded to float,
 * every operation is a float operation in the fixed fma order above, and the
 * result is widened back to double.  Factors are given as doubles holding
 * float values. */
void or_lsolve_f32(int32_t nx, int32_t ny, const double *lw, const double *ls,
                   const double *q, double *y) {
  const size_t n = (size_t)nx * (size_t)ny;
  float *yf = malloc(sizeof(float) * (n ? n : 1));
  for (size_t k = 0; k < n; ++k) {
    const int32_t i = (int32_t)(k % (size_t)nx);
    const int32_t j = (int32_t)(k / (size_t)nx);
    const float yw = (i > 0) ? yf[k - 1] : 0.0f;
    const float ys = (j > 0) ? yf[k - nx] : 0.0f;
    float t = fmaf(-(float)lw[k], yw, (float)q[k]);
    t = fmaf(-(float)ls[k], ys, t);
    yf[k] = t;
    y[k] = (double)t;
  }
  free(yf);
}

void or_usolve_f32(int32_t nx, int32_t ny, const double *ue, const double *un,
                   const double *invd, const double *y, double *z) {
  const size_t n = (size_t)nx * (size_t)ny;
  float *zf = malloc(sizeof(float) * (n ? n : 1));
  for (size_t kk = n; kk-- > 0;) {
    const int32_t i = (int32_t)(kk % (size_t)nx);
    const int32_t j = (int32_t)(kk / (size_t)nx);
    const float ze = (i < nx - 1) ? zf[kk + 1] : 0.0f;
    const float zn = (j < ny - 1) ? zf[kk + nx] : 0.0f;
    float t = fmaf(-(float)ue[kk], ze, (float)y[kk]);
    t = fmaf(-(float)un[kk], zn, t);
    t = t * (float)invd[kk];
    zf[kk] = t;
    z[kk] = (double)t;
  }
  free(zf);
}

/* ------------------------------------------------------------------------ */
/* Inner products in double-double arithmetic.                              */
/* ------------------------------------------------------------------------ */
/* Error-free transformations (Knuth's TwoSum, Dekker's FastTwoSum, TwoProd by
 * fma) and the accurate double-word addition of Joldes, Muller & Popescu
 * (ACM TOMS 44(2), 2017, "AccurateDWPlusDW").  The dot product accumulates
 * every exact product x_k*y_k = p + e in double-double, in index order, and
 * returns the high word: the result is the exact dot product rounded to
 * nearest up to an error of order n*u^2*sum|x_k y_k|, so it does not depend
 * on the order of summation except in near-tie cases. */
typedef struct { double hi, lo; } or_dd;

static inline void two_sum(double a, double b, double *s, double *e) {
  const double ss = a + b;
  const double bb = ss - a;
  *e = (a - (ss - bb)) + (b - bb);
  *s = ss;
}
static inline void fast_two_sum(double a, double b, double *s, double *e) {
  const double ss = a + b;
  *e = b - (ss - a);
  *s = ss;
}
static inline or_dd dd_add(or_dd x, or_dd y) {
  double sh, sl, th, tl, vh, vl, zh, zl;
  two_sum(x.hi, y.hi, &sh, &sl);
  two_sum(x.lo, y.lo, &th, &tl);
  const double c = sl + th;
  fast_two_sum(sh, c, &vh, &vl);
  const double w = tl + vl;
  fast_two_sum(vh, w, &zh, &zl);
  or_dd z = {zh, zl};
  return z;
}

double or_dot(int64_t n, const double *x, const double *y) {
  or_dd s = {0.0, 0.0};
  for (int64_t k = 0; k < n; ++k) {
    const double p = x[k] * y[k];
    const double e = fma(x[k], y[k], -p);
    or_dd t = {p, e};
    s = dd_add(s, t);
  }
  return s.hi;
}

double or_maxabs(int64_t n, const double *x) {
  /* max |x_k|; a NaN anywhere makes the result NaN */
  double m = 0.0;
  for (int64_t k = 0; k < n; ++k) {
    const double v = fabs(x[k]);
    if (isnan(v)) return v;
    if (v > m) m = v;
  }
  return m;
}

/* ------------------------------------------------------------------------ */
/* Section 5.2: preconditioned BiCGSTAB.                                    */
/* ------------------------------------------------------------------------ */

/* Result record of one solve. */
typedef struct {
  int32_t status;      /* OR_OK, OR_MAXIT, OR_BREAKDOWN_RHO, OR_OMEGA_ZERO, OR_NONFINITE, OR_INACCURATE */
  int32_t iters;       /* loop passes started (a half-step exit counts) */
  int32_t hist_len;    /* valid entries of the residual histories */
  int32_t half_step;   /* 1 if the last pass ended on the ||s|| test */
  double bnorm;        /* ||b||_2 */
  double true_relres;  /* ||b - A x||_2 / ||b||_2 at exit (0 when b = 0) */
  int32_t restarts;    /* restarts from the current iterate (see below) */
  int32_t pad;
} or_solve_info;

/* Apply M^{-1} = U^{-1} L^{-1} (double or single precision substitutions). */
static void apply_precond(int32_t nx, int32_t ny, const double *lw, const double *ls,
                          const double *ue, const double *un, const double *invd,
                          int32_t sweep_f32, const double *q, double *tmp, double *out) {
  if (sweep_f32) {
    or_lsolve_f32(nx, ny, lw, ls, q, tmp);
    or_usolve_f32(nx, ny, ue, un, invd, tmp, out);
  } else {
    or_lsolve(nx, ny, lw, ls, q, tmp);
    or_usolve(nx, ny, ue, un, invd, tmp, out);
  }
}

/* e = b - A x by plain subtraction; returns ||e||_2 (double-double dot). */
static double true_residual(int32_t nx, int32_t ny, const double *S, const double *W,
                            const double *C, const double *E, const double *N,
                            const double *b, const double *x, double *tmp, double *e) {
  const int64_t n = (int64_t)nx * (int64_t)ny;
  or_spmv(nx, ny, S, W, C, E, N, x, tmp);
  for (int64_t k = 0; k < n; ++k) e[k] = b[k] - tmp[k];
  return sqrt(or_dot(n, e, e));
}

/* Right-preconditioned BiCGSTAB as the algorithm of Section 5.2 (and its
 * appendix implementation): r0 = b - A x0, r^ = r0; per pass i:
 *   rho = r^.r (fail on 0); p = r (first pass) or
 *   p = r + beta (p - omega v), beta = (rho_i/rho_{i-1}) (alpha/omega);
 *   M p^ = p; v = A p^; alpha = rho / (r^.v); s = r - alpha v;
 *   if ||s|| small: x += alpha p^, converged;
 *   M z = s; t = A z; omega = (t.s)/(t.t); x += alpha p^ + omega z;
 *   r = s - omega t; record ||r||; converged if ||r|| small; stop if omega = 0.
 * M = L U with L = I + (lw, ls) and U = diag(1/invd) + (ue, un).
 * Stopping ("small"): ||.||_2 < tol*||b||_2 (abs_tol = 0) or ||.||_2 < tol
 * (abs_tol = 1, the appendix's absolute test).  If ||r0|| already passes the
 * test the solve returns with zero passes.  b = 0 returns x = 0.
 *
 * The tests above look at the recursively updated residual, which can drift
 * away from the true residual b - A x (the paper is silent on this).  With
 * max_restarts >= 0 a convergence of the recursion is accepted only if the
 * true residual passes the same test; otherwise, if passes are left
 * (i < maxit) and fewer than max_restarts restarts were made, the method
 * starts again from the current iterate as from an initial guess
 * (r = r^ = b - A x, next pass with p = r), else it stops with OR_MAXIT
 * (i = maxit) or OR_INACCURATE.  max_restarts < 0 keeps the recursive test
 * alone (the appendix's behaviour).
 *
 * Fixed update formulas: p = fma(beta, fma(-omega, v, p), r),
 * s = fma(-alpha, v, r), x = fma(omega, z, fma(alpha, p^, x)),
 * r = fma(-omega, t, s); r0 = b - A x0 (and b - A x at a check) by plain
 * subtraction.
 * sweep_f32 = 1 applies M^{-1} with the single-precision substitutions
 * (or_lsolve_f32 / or_usolve_f32); the factors must then hold float values.
 * x0 may be NULL (zero guess).  hist_l2/hist_max hold maxit+1 entries:
 * entry 0 is ||r0||, entry i the recursively updated ||r_i|| after pass i, or
 * ||s|| at a half-step exit. */
int or_bicgstab(int32_t nx, int32_t ny,
                const double *S, const double *W, const double *C, const double *E, const double *N,
                const double *lw, const double *ls, const double *invd,
                const double *ue, const double *un,
                const double *b, const double *x0, double tol, int32_t abs_tol, int32_t maxit,
                int32_t sweep_f32, int32_t max_restarts,
                double *x, double *hist_l2, double *hist_max, or_solve_info *info) {
  const int64_t n = (int64_t)nx * (int64_t)ny;
  memset(info, 0, sizeof(*info));
  if (nx < 1 || ny < 1 || maxit < 0 || !(tol >= 0.0)) {
    info->status = OR_ERR_ARG;
    return OR_ERR_ARG;
  }
  double *r = calloc((size_t)n, sizeof(double)), *rh = calloc((size_t)n, sizeof(double));
  double *p = calloc((size_t)n, sizeof(double)), *v = calloc((size_t)n, sizeof(double));
  double *s = calloc((size_t)n, sizeof(double)), *t = calloc((size_t)n, sizeof(double));
  double *ph = calloc((size_t)n, sizeof(double)), *z = calloc((size_t)n, sizeof(double));
  double *yy = calloc((size_t)n, sizeof(double));
  int status = OR_MAXIT;
  int32_t it = 0, hl = 0, restarts = 0, half = 0;
  const double bnorm = sqrt(or_dot(n, b, b));
  info->bnorm = bnorm;
  if (x0) memcpy(x, x0, sizeof(double) * (size_t)n);
  else memset(x, 0, sizeof(double) * (size_t)n);
  if (bnorm == 0.0) {
    memset(x, 0, sizeof(double) * (size_t)n);
    if (hist_l2) { hist_l2[0] = 0.0; hist_max[0] = 0.0; }
    info->status = OR_OK; info->iters = 0; info->hist_len = 1; info->true_relres = 0.0;
    goto done;
  }
  const double thr = abs_tol ? tol : tol * bnorm;
  /* r0 = b - A x0 */
  double rnorm = true_residual(nx, ny, S, W, C, E, N, b, x, v, r);
  memcpy(rh, r, sizeof(double) * (size_t)n);
  hist_l2[0] = rnorm;
  hist_max[0] = or_maxabs(n, r);
  hl = 1;
  if (!isfinite(rnorm)) { status = OR_NONFINITE; goto finish; }
  if (rnorm < thr) { status = OR_OK; goto finish; }
  double rho = or_dot(n, rh, r), rho_prev = 0.0, alpha = 0.0, omega = 0.0;
  int fresh = 1;   /* p = r: the first pass and the first pass after a restart */
  for (int32_t i = 1; i <= maxit; ++i) {
    it = i;
    if (!isfinite(rho)) { status = OR_NONFINITE; break; }
    if (rho == 0.0) { status = OR_BREAKDOWN_RHO; break; }
    if (fresh) {
      memcpy(p, r, sizeof(double) * (size_t)n);
    } else {
      const double beta = (rho / rho_prev) * (alpha / omega);
      for (int64_t k = 0; k < n; ++k) p[k] = fma(beta, fma(-omega, v[k], p[k]), r[k]);
    }
    fresh = 0;
    apply_precond(nx, ny, lw, ls, ue, un, invd, sweep_f32, p, yy, ph);
    or_spmv(nx, ny, S, W, C, E, N, ph, v);
    alpha = rho / or_dot(n, rh, v);
    if (!isfinite(alpha)) { status = OR_NONFINITE; break; }
    for (int64_t k = 0; k < n; ++k) s[k] = fma(-alpha, v[k], r[k]);
    const double snorm = sqrt(or_dot(n, s, s));
    if (!isfinite(snorm)) { status = OR_NONFINITE; break; }
    int converged = 0;
    if (snorm < thr) {
      for (int64_t k = 0; k < n; ++k) x[k] = fma(alpha, ph[k], x[k]);
      hist_l2[i] = snorm;
      hist_max[i] = or_maxabs(n, s);
      hl = i + 1;
      half = 1;
      converged = 1;
    } else {
      apply_precond(nx, ny, lw, ls, ue, un, invd, sweep_f32, s, yy, z);
      or_spmv(nx, ny, S, W, C, E, N, z, t);
      const double ts = or_dot(n, t, s), tt = or_dot(n, t, t);
      omega = ts / tt;
      if (!isfinite(omega)) { status = OR_NONFINITE; break; }
      for (int64_t k = 0; k < n; ++k) {
        x[k] = fma(omega, z[k], fma(alpha, ph[k], x[k]));
        r[k] = fma(-omega, t[k], s[k]);
      }
      rnorm = sqrt(or_dot(n, r, r));
      hist_l2[i] = rnorm;
      hist_max[i] = or_maxabs(n, r);
      hl = i + 1;
      rho_prev = rho;
      rho = or_dot(n, rh, r);
      if (!isfinite(rnorm)) { status = OR_NONFINITE; break; }
      if (rnorm < thr) converged = 1;
      else if (omega == 0.0) { status = OR_OMEGA_ZERO; break; }
    }
    if (converged) {
      if (max_restarts < 0) { status = OR_OK; break; }
      /* the recursion converged: check the true residual */
      const double te = true_residual(nx, ny, S, W, C, E, N, b, x, v, t);
      if (te < thr) { status = OR_OK; break; }
      if (i >= maxit) { status = OR_MAXIT; break; }
      if (restarts >= max_restarts) { status = OR_INACCURATE; break; }
      /* restart from the current iterate: r = r^ = b - A x */
      ++restarts;
      half = 0;
      memcpy(r, t, sizeof(double) * (size_t)n);
      memcpy(rh, t, sizeof(double) * (size_t)n);
      rho = or_dot(n, rh, r);
      fresh = 1;
    }
  }
finish:
  info->status = status;
  info->iters = it;
  info->hist_len = hl;
  info->half_step = half;
  info->restarts = restarts;
  /* true residual at exit */
  info->true_relres = true_residual(nx, ny, S, W, C, E, N, b, x, v, t) / bnorm;
done:
  free(r); free(rh); free(p); free(v); free(s); free(t); free(ph); free(z); free(yy);
  return info->status;
}

/* Post-processing of the appendix drivers: the full (nx+2) x (ny+2) grid
 * (row-major, x fastest) with Dirichlet edges from the exact u, Neumann edges
 * reconstructed as U(X,y) = U(x_nx,y) + dx g_x(y), U(x,Y) = U(x,y_ny) + dy g_y(x)
 * and the corner from the x-direction, U(X,Y) = U(x_nx,Y) + dx g_x(Y).
 * Returns max |U - u_exact| over all nodes. */
double or_max_error(double X, double Y, int32_t nx, int32_t ny, int32_t bc,
                    const double *sol, double *grid) {
  const int32_t mx = nx + 2, my = ny + 2;
  const double dx = X / (double)(nx + 1), dy = Y / (double)(ny + 1);
  double *U = grid ? grid : malloc(sizeof(double) * (size_t)mx * (size_t)my);
  for (int32_t jj = 0; jj < my; ++jj)
    for (int32_t ii = 0; ii < mx; ++ii) {
      const double xx = (double)ii * dx, yy = (double)jj * dy;
      U[(size_t)jj * mx + ii] = or_u_exact(xx, yy, X, Y);
    }
  U[0] = 0.0;
  for (int32_t ii = 0; ii < mx; ++ii) U[ii] = 0.0; /* y = 0: u = 0 */
  for (int32_t j = 0; j < ny; ++j)
    for (int32_t i = 0; i < nx; ++i)
      U[(size_t)(j + 1) * mx + (i + 1)] = sol[(size_t)j * nx + i];
  if (bc == 1) {
    const double e1 = exp(-1.0);
    for (int32_t jj = 1; jj <= ny + 1; ++jj) {
      const double yy = (double)jj * dy;
      const double gxv = (((-1.0 / X) * e1) * (1.0 - exp(-yy / Y))) * yy;
      if (jj <= ny) U[(size_t)jj * mx + (nx + 1)] = U[(size_t)jj * mx + nx] + dx * gxv;
    }
    for (int32_t ii = 1; ii <= nx; ++ii) {
      const double xx = (double)ii * dx;
      const double gyv = exp(-xx / X) * (e1 + (1.0 - e1));
      U[(size_t)(ny + 1) * mx + ii] = U[(size_t)ny * mx + ii] + dy * gyv;
    }
    const double gxc = (((-1.0 / X) * e1) * (1.0 - exp(-1.0))) * Y;
    U[(size_t)(ny + 1) * mx + (nx + 1)] = U[(size_t)(ny + 1) * mx + nx] + dx * gxc;
  }
  double err = 0.0;
  for (int32_t jj = 0; jj < my; ++jj)
    for (int32_t ii = 0; ii < mx; ++ii) {
      const double xx = (double)ii * dx, yy = (double)jj * dy;
      const double e = fabs(U[(size_t)jj * mx + ii] - or_u_exact(xx, yy, X, Y));
      if (e > err) err = e;
    }
  if (!grid) free(U);
  return err;
}
