/*
 * wave_oracle.c -- FP64 CPU oracle for the dimensionally unsplit
 * wave-propagation step of 2D linear acoustics
 * (Qin, LeVeque & Motley, arXiv 1808.02638).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark load it; the
 * product path never links, imports or calls it, and it shares no code,
 * header, table or constant with the GPU library.
 *
 * What it follows:
 *   - the update formula, paper Sec. 2.1 eq. (2.3): first-order fluctuations
 *     A+dQ, A-dQ, B+dQ, B-dQ plus the differences of the second-order
 *     correction fluxes F~ and G~, which hold both the limited-wave
 *     corrections and the transverse waves obtained by splitting the
 *     fluctuations in the other direction (Sec. 2.1, last paragraph, and
 *     Sec. 3.3, "normal and transverse Riemann solvers");
 *   - the acoustics system q = (p,u,v), q_t + A q_x + B q_y = 0 with the
 *     matrices of Sec. 4.1 eqs. (4.1)-(4.2);
 *   - the Courant number of Sec. 2.4 eq. (2.10) and the time-step rule of
 *     Sec. 2.5 eq. (2.11) (applied by the Python driver);
 *   - physical boundaries through ghost cells, Sec. 2.2 item 1; the benchmark
 *     uses non-reflecting outflow (Sec. 4.1), i.e. zero-order extrapolation.
 * The paper defers the exact form of the correction terms to LeVeque's
 * finite-volume book (its standard unsplit wave-propagation method with
 * transverse Riemann solvers); the readings taken where the paper is silent
 * are listed in the repository design notes:
 *   * the transverse solver splits the first-order fluctuations; with
 *     OR_OPT_TRANSVERSE_CORR it first moves each edge's whole limited
 *     correction sum_p |s_p| (1 - |s_p| dt/dx) W~_p into them (the sign and an
 *     upper bound on that amount are pinned by stability; the amount itself,
 *     all of it rather than half, is parity unpinned);
 *   * limiter ratio theta = (W_upwind . W) / (W . W) over all components,
 *     W~ = W when W . W = 0; MC limiter phi = max(0, min((1+theta)/2, 2, 2 theta));
 *   * CFL number of a 2D step = max over x-edges of |s| dt/dx and over
 *     y-edges of |s| dt/dy.
 *
 * Everything is written edge by edge with explicit arrays for the
 * fluctuations and for F~ and G~, with all three eigen-waves (speeds -c, 0,
 * +c) taken from the full eigen-decomposition.  OpenMP parallelises rows /
 * columns (each writes only its own entries) and independent patches.
 *
 * Storage of one patch: dense [3][my+4][mx+4] doubles (components p, u, v;
 * two ghost layers on every side; x fastest).  Interior cells are
 * i = 0..mx-1, j = 0..my-1; ghost cells are i = -2,-1,mx,mx+1 (and j alike).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NM 3 /* components of q = (p, u, v) */
#define NW 3 /* waves: eigenvalues -c, 0, +c */

enum { OR_LIM_MC = 0, OR_LIM_NONE = 1, OR_LIM_ZERO = 2, OR_LIM_VANLEER = 3 };
enum { OR_BC_EXTRAP = 0, OR_BC_PERIODIC = 1 };
enum { OR_OPT_DROP_ZERO_WAVE = 1, OR_OPT_TRANSVERSE_CORR = 2 };

/* ---------------------------------------------------------------------- */
/* Eigen-decomposition of A (dir 0) and B (dir 1), Sec. 4.1 eq. (4.2).      */
/* ---------------------------------------------------------------------- */
typedef struct {
  double s[NW];     /* eigenvalues, ordered -c, 0, +c              */
  double R[NM][NW]; /* right eigenvectors, one per column          */
  double L[NW][NM]; /* left eigenvectors (rows of R^-1)            */
} eig_t;

static void acoustics_eig(double rho, double K, int dir, eig_t *e) {
  const double c = sqrt(K / rho); /* sound speed c = sqrt(K0/rho0) */
  const double Z = rho * c;       /* impedance                      */
  const int n = (dir == 0) ? 1 : 2; /* normal velocity component     */
  const int t = (dir == 0) ? 2 : 1; /* tangential velocity component */
  memset(e, 0, sizeof *e);
  e->s[0] = -c;
  e->s[1] = 0.0;
  e->s[2] = c;
  /* r^(-c) = (-Z, e_n), r^(0) = e_t, r^(+c) = (Z, e_n) */
  e->R[0][0] = -Z;
  e->R[n][0] = 1.0;
  e->R[t][1] = 1.0;
  e->R[0][2] = Z;
  e->R[n][2] = 1.0;
  /* alpha^(-c) = (-dp + Z dn)/(2Z), alpha^(0) = dt, alpha^(+c) = (dp + Z dn)/(2Z) */
  e->L[0][0] = -1.0 / (2.0 * Z);
  e->L[0][n] = 0.5;
  e->L[1][t] = 1.0;
  e->L[2][0] = 1.0 / (2.0 * Z);
  e->L[2][n] = 0.5;
}

/* Normal Riemann solve at one edge: waves W^p = alpha^p r^p with
 * alpha = R^-1 (q_r - q_l), and fluctuations A-dQ = sum_{s<0} s W,
 * A+dQ = sum_{s>0} s W.  drop_zero_wave omits the speed-0 wave. */
static void riemann(const eig_t *e, const double ql[NM], const double qr[NM],
                    int drop_zero_wave, double wave[NW][NM], double amdq[NM],
                    double apdq[NM]) {
  double dq[NM], alpha[NW];
  for (int m = 0; m < NM; ++m) dq[m] = qr[m] - ql[m];
  for (int p = 0; p < NW; ++p) {
    alpha[p] = 0.0;
    for (int m = 0; m < NM; ++m) alpha[p] += e->L[p][m] * dq[m];
    if (drop_zero_wave && e->s[p] == 0.0) alpha[p] = 0.0;
  }
  for (int p = 0; p < NW; ++p)
    for (int m = 0; m < NM; ++m) wave[p][m] = alpha[p] * e->R[m][p];
  for (int m = 0; m < NM; ++m) amdq[m] = apdq[m] = 0.0;
  for (int p = 0; p < NW; ++p) {
    if (drop_zero_wave && e->s[p] == 0.0) continue;
    for (int m = 0; m < NM; ++m) {
      if (e->s[p] < 0.0) amdq[m] += e->s[p] * wave[p][m];
      else if (e->s[p] > 0.0) apdq[m] += e->s[p] * wave[p][m];
    }
  }
}

/* Transverse Riemann solve: split a vector a by the other direction's
 * eigen-structure into its negative- and positive-speed parts. */
static void split(const eig_t *e, const double a[NM], double minus[NM],
                  double plus[NM]) {
  double beta[NW];
  for (int p = 0; p < NW; ++p) {
    beta[p] = 0.0;
    for (int m = 0; m < NM; ++m) beta[p] += e->L[p][m] * a[m];
  }
  for (int m = 0; m < NM; ++m) minus[m] = plus[m] = 0.0;
  for (int p = 0; p < NW; ++p)
    for (int m = 0; m < NM; ++m) {
      if (e->s[p] < 0.0) minus[m] += e->s[p] * beta[p] * e->R[m][p];
      else if (e->s[p] > 0.0) plus[m] += e->s[p] * beta[p] * e->R[m][p];
    }
}

/* ---------------------------------------------------------------------- */
/* Wave limiter                                                            */
/* ---------------------------------------------------------------------- */
double oracle_phi(int lim, double theta) {
  switch (lim) {
  case OR_LIM_MC:
    return fmax(0.0, fmin(fmin(0.5 * (1.0 + theta), 2.0), 2.0 * theta));
  case OR_LIM_NONE:
    return 1.0;
  case OR_LIM_ZERO:
    return 0.0;
  case OR_LIM_VANLEER:
    return (theta + fabs(theta)) / (1.0 + fabs(theta));
  }
  return NAN;
}

/* Branch of the MC limiter taken at ratio theta:
 * 0 -> phi = 0, 1 -> (1+theta)/2, 2 -> 2, 3 -> 2 theta; ties go to the
 * lowest index.  A zero wave (W.W = 0) is branch 0. */
int oracle_mc_branch(double ww, double theta) {
  if (ww == 0.0 || theta <= 0.0) return 0;
  const double b1 = 0.5 * (1.0 + theta), b2 = 2.0, b3 = 2.0 * theta;
  if (b1 <= b2 && b1 <= b3) return 1;
  if (b2 <= b3) return 2;
  return 3;
}

static double dot3(const double a[NM], const double b[NM]) {
  double s = 0.0;
  for (int m = 0; m < NM; ++m) s += a[m] * b[m];
  return s;
}

/* Limited wave W~ from W and its upwind neighbour.  With a frozen branch
 * (frozen >= 0) the map is the linear one that branch selects:
 * 0 -> 0, 1 -> (W + W_up)/2, 2 -> 2 W, 3 -> 2 W_up. */
static void limit_wave(int lim, const double w[NM], const double wup[NM],
                       int frozen, double out[NM], int *branch) {
  if (frozen >= 0) {
    for (int m = 0; m < NM; ++m) {
      switch (frozen) {
      case 0: out[m] = 0.0; break;
      case 1: out[m] = 0.5 * (w[m] + wup[m]); break;
      case 2: out[m] = 2.0 * w[m]; break;
      default: out[m] = 2.0 * wup[m]; break;
      }
    }
    if (branch) *branch = frozen;
    return;
  }
  const double ww = dot3(w, w);
  if (ww == 0.0) {
    for (int m = 0; m < NM; ++m) out[m] = w[m];
    if (branch) *branch = 0;
    return;
  }
  const double theta = dot3(wup, w) / ww;
  const double f = oracle_phi(lim, theta);
  for (int m = 0; m < NM; ++m) out[m] = f * w[m];
  if (branch) *branch = oracle_mc_branch(ww, theta);
}

/* ---------------------------------------------------------------------- */
/* Indexing                                                                */
/* ---------------------------------------------------------------------- */
#define QIX(m, i, j)                                                           \
  ((((size_t)(m) * (size_t)(my + 4) + (size_t)((j) + 2)) * (size_t)(mx + 4)) + \
   (size_t)((i) + 2))

/* mask byte of cell (i,j), i in [0,mx], j in [0,my]:
 *   bits 0-1 x-edge (i-1/2, j) wave -c, bits 2-3 x-edge wave +c,
 *   bits 4-5 y-edge (i, j-1/2) wave -c, bits 6-7 y-edge wave +c. */
#define MIX(i, j) ((size_t)(j) * (size_t)(mx + 1) + (size_t)(i))

/* ---------------------------------------------------------------------- */
/* Boundary conditions (Sec. 2.2 item 1; outflow = zero-order extrapolation) */
/* ---------------------------------------------------------------------- */
/* x-ghosts for the interior rows first, then y-ghosts across the full padded
 * width, so the corner ghosts take the value of the nearest interior cell. */
void oracle_fill_bc(double *q, int mx, int my, int bc_kind) {
  for (int m = 0; m < NM; ++m) {
    for (int j = 0; j < my; ++j)
      for (int g = 1; g <= 2; ++g) {
        if (bc_kind == OR_BC_PERIODIC) {
          q[QIX(m, -g, j)] = q[QIX(m, mx - g, j)];
          q[QIX(m, mx - 1 + g, j)] = q[QIX(m, g - 1, j)];
        } else {
          q[QIX(m, -g, j)] = q[QIX(m, 0, j)];
          q[QIX(m, mx - 1 + g, j)] = q[QIX(m, mx - 1, j)];
        }
      }
    for (int i = -2; i < mx + 2; ++i)
      for (int g = 1; g <= 2; ++g) {
        if (bc_kind == OR_BC_PERIODIC) {
          q[QIX(m, i, -g)] = q[QIX(m, i, my - g)];
          q[QIX(m, i, my - 1 + g)] = q[QIX(m, i, g - 1)];
        } else {
          q[QIX(m, i, -g)] = q[QIX(m, i, 0)];
          q[QIX(m, i, my - 1 + g)] = q[QIX(m, i, my - 1)];
        }
      }
  }
}

/* ---------------------------------------------------------------------- */
/* One unsplit step of one patch                                           */
/* ---------------------------------------------------------------------- */
/*
 * q_in, q_out : dense [3][my+4][mx+4]; q_out's interior receives Q^{n+1},
 *               its ghosts are copied from q_in (the boundary fill is a
 *               separate call the caller makes between steps).
 * limiter     : OR_LIM_*.
 * options     : OR_OPT_* bits.  OR_OPT_DROP_ZERO_WAVE omits the speed-0
 *               wave.  OR_OPT_TRANSVERSE_CORR selects the variant whose
 *               transverse solver also splits the limited second-order
 *               correction (the correction waves are propagated
 *               transversely); the update itself is unchanged.
 * frozen      : NULL, or (mx+1)*(my+1) mask bytes fixing the MC branches
 *               (the step is then a linear map of q_in);
 * masks_out   : NULL, or (mx+1)*(my+1) bytes receiving the branches taken.
 *               Neither mask argument is accepted with OR_OPT_TRANSVERSE_CORR
 *               (that variant also limits on the two outer ghost rows and
 *               columns, which have no mask bytes).
 * cfl_out     : max over edges of |s| dt/dx (x-edges) and |s| dt/dy (y-edges).
 * Returns 0, or -1 on bad sizes / allocation failure.
 */
/* Optional outputs of the step: the terms of eq. (2.3) at every edge of the
 * interior cells, as the update uses them.
 *   x-edges (i-1/2, j), j = 0..my-1, i = 0..mx: [my][mx+1][3]
 *     Fx  = F~ (normal correction plus transverse contributions),
 *     amx = A-dQ, apx = A+dQ;
 *   y-edges (i, j-1/2), j = 0..my, i = 0..mx-1: [my+1][mx][3]
 *     Gy = G~, amy = B-dQ, apy = B+dQ. */
typedef struct {
  double *Fx, *amx, *apx, *Gy, *amy, *apy;
} edge_terms_t;

static int step_core(const double *q_in, double *q_out, int mx, int my,
                     double dx, double dy, double dt, double rho, double K,
                     int limiter, int options, const uint8_t *frozen,
                     uint8_t *masks_out, double *cfl_out, int parallel,
                     const edge_terms_t *terms) {
  if (mx < 1 || my < 1 || !(dx > 0.0) || !(dy > 0.0)) return -1;
  const int drop_zero_wave = (options & OR_OPT_DROP_ZERO_WAVE) != 0;
  const int tcorr = (options & OR_OPT_TRANSVERSE_CORR) != 0;
  if (tcorr && (frozen || masks_out)) return -1;
  eig_t ex, ey;
  acoustics_eig(rho, K, 0, &ex);
  acoustics_eig(rho, K, 1, &ey);
  const double dtdx = dt / dx, dtdy = dt / dy;
  const int par = parallel && ((long)mx * (long)my >= 16384);

  /* x-edge arrays: rows j = -1..my, edges e = 0..mx (edge e is i-1/2 of cell e) */
  const size_t nxe = (size_t)(my + 2) * (size_t)(mx + 1);
  /* y-edge arrays: edges f = 0..my, columns i = -1..mx */
  const size_t nye = (size_t)(my + 1) * (size_t)(mx + 2);
  double *amdq_x = calloc(nxe * NM, sizeof(double));
  double *apdq_x = calloc(nxe * NM, sizeof(double));
  double *amdq_y = calloc(nye * NM, sizeof(double));
  double *apdq_y = calloc(nye * NM, sizeof(double));
  /* normal-direction corrections: F at (rows 0..my-1, edges 0..mx),
   * G at (edges 0..my, columns 0..mx-1) */
  double *Fc = calloc((size_t)my * (mx + 1) * NM, sizeof(double));
  double *Gc = calloc((size_t)(my + 1) * mx * NM, sizeof(double));
  /* transverse contributions, stored per cell they originate from:
   * Gx_top/Gx_bot: from the x-fluctuations entering cell (i,j), to G~ at
   *   (i, j+1/2) / (i, j-1/2); cells i = 0..mx-1, j = -1..my.
   * Fy_right/Fy_left: from the y-fluctuations entering cell (i,j), to F~ at
   *   (i+1/2, j) / (i-1/2, j); cells i = -1..mx, j = 0..my-1. */
  double *Gx_top = calloc((size_t)(my + 2) * mx * NM, sizeof(double));
  double *Gx_bot = calloc((size_t)(my + 2) * mx * NM, sizeof(double));
  double *Fy_right = calloc((size_t)my * (mx + 2) * NM, sizeof(double));
  double *Fy_left = calloc((size_t)my * (mx + 2) * NM, sizeof(double));
  int rc = 0;
  if (masks_out) memset(masks_out, 0, (size_t)(mx + 1) * (size_t)(my + 1));
  if (!amdq_x || !apdq_x || !amdq_y || !apdq_y || !Fc || !Gc || !Gx_top ||
      !Gx_bot || !Fy_right || !Fy_left) {
    rc = -1;
    goto done;
  }

#define AX(j, e) (((size_t)((j) + 1) * (size_t)(mx + 1) + (size_t)(e)) * NM)
#define AY(f, i) (((size_t)(f) * (size_t)(mx + 2) + (size_t)((i) + 1)) * NM)
#define FC(j, e) (((size_t)(j) * (size_t)(mx + 1) + (size_t)(e)) * NM)
#define GC(f, i) (((size_t)(f) * (size_t)mx + (size_t)(i)) * NM)
#define GX(j, i) (((size_t)((j) + 1) * (size_t)mx + (size_t)(i)) * NM)
#define FY(j, i) (((size_t)(j) * (size_t)(mx + 2) + (size_t)((i) + 1)) * NM)

  /* ---- x-direction: rows j = -1..my ---- */
#pragma omp parallel for if (par) schedule(static)
  for (int j = -1; j <= my; ++j) {
    /* waves at edges e = -1..mx+1 of this row (the outer two feed the
     * limiter only) */
    double(*w)[NW][NM] = malloc(sizeof(double[NW][NM]) * (size_t)(mx + 3));
    for (int e = -1; e <= mx + 1; ++e) {
      double ql[NM], qr[NM], am[NM], ap[NM];
      for (int m = 0; m < NM; ++m) {
        ql[m] = q_in[QIX(m, e - 1, j)];
        qr[m] = q_in[QIX(m, e, j)];
      }
      riemann(&ex, ql, qr, drop_zero_wave, w[e + 1], am, ap);
      if (e >= 0 && e <= mx)
        for (int m = 0; m < NM; ++m) {
          amdq_x[AX(j, e) + m] = am[m];
          apdq_x[AX(j, e) + m] = ap[m];
        }
    }
    /* limited-wave correction flux: the normal part of F~ on interior rows;
     * the transverse variant needs it on the ghost rows -1 and my too */
    double(*F)[NM] = calloc((size_t)(mx + 1), sizeof(double[NM]));
    const int interior = (j >= 0 && j < my);
    if (interior || tcorr)
      for (int e = 0; e <= mx; ++e) {
        int mask_bits = 0;
        for (int p = 0; p < NW; ++p) {
          const double s = ex.s[p];
          const int up = (s > 0.0) ? e - 1 : (s < 0.0 ? e + 1 : e);
          int fz = -1, br = 0;
          if (frozen && s != 0.0)
            fz = (frozen[MIX(e, j)] >> (p == 0 ? 0 : 2)) & 3;
          double wl[NM];
          limit_wave(limiter, w[e + 1][p], w[up + 1][p], fz, wl, &br);
          if (s != 0.0) mask_bits |= br << (p == 0 ? 0 : 2);
          const double coef = 0.5 * fabs(s) * (1.0 - dtdx * fabs(s));
          for (int m = 0; m < NM; ++m) F[e][m] += coef * wl[m];
        }
        if (interior) {
          for (int m = 0; m < NM; ++m) Fc[FC(j, e) + m] = F[e][m];
          if (masks_out) masks_out[MIX(e, j)] = (uint8_t)mask_bits;
        }
      }
    /* transverse: A+dQ at edge e enters cell e, A-dQ enters cell e-1.  The
     * variant first moves the correction into them: A+dQ - 2F, A-dQ + 2F
     * (2F = sum_p |s_p| (1 - |s_p| dt/dx) W~_p; their sum is still A dQ). */
    for (int e = 0; e <= mx; ++e) {
      double ap[NM], am[NM], bm[NM], bp[NM];
      for (int m = 0; m < NM; ++m) {
        ap[m] = apdq_x[AX(j, e) + m];
        am[m] = amdq_x[AX(j, e) + m];
        if (tcorr) {
          ap[m] -= 2.0 * F[e][m];
          am[m] += 2.0 * F[e][m];
        }
      }
      if (e <= mx - 1) {
        split(&ey, ap, bm, bp);
        for (int m = 0; m < NM; ++m) {
          Gx_top[GX(j, e) + m] -= 0.5 * dtdx * bp[m];
          Gx_bot[GX(j, e) + m] -= 0.5 * dtdx * bm[m];
        }
      }
      if (e >= 1) {
        split(&ey, am, bm, bp);
        for (int m = 0; m < NM; ++m) {
          Gx_top[GX(j, e - 1) + m] -= 0.5 * dtdx * bp[m];
          Gx_bot[GX(j, e - 1) + m] -= 0.5 * dtdx * bm[m];
        }
      }
    }
    free(F);
    free(w);
  }

  /* ---- y-direction: columns i = -1..mx ---- */
#pragma omp parallel for if (par) schedule(static)
  for (int i = -1; i <= mx; ++i) {
    double(*w)[NW][NM] = malloc(sizeof(double[NW][NM]) * (size_t)(my + 3));
    for (int f = -1; f <= my + 1; ++f) {
      double ql[NM], qr[NM], bm[NM], bp[NM];
      for (int m = 0; m < NM; ++m) {
        ql[m] = q_in[QIX(m, i, f - 1)];
        qr[m] = q_in[QIX(m, i, f)];
      }
      riemann(&ey, ql, qr, drop_zero_wave, w[f + 1], bm, bp);
      if (f >= 0 && f <= my)
        for (int m = 0; m < NM; ++m) {
          amdq_y[AY(f, i) + m] = bm[m];
          apdq_y[AY(f, i) + m] = bp[m];
        }
    }
    /* normal part of G~ on interior columns (all columns for the variant) */
    double(*G)[NM] = calloc((size_t)(my + 1), sizeof(double[NM]));
    const int interior = (i >= 0 && i < mx);
    if (interior || tcorr)
      for (int f = 0; f <= my; ++f) {
        int mask_bits = 0;
        for (int p = 0; p < NW; ++p) {
          const double s = ey.s[p];
          const int up = (s > 0.0) ? f - 1 : (s < 0.0 ? f + 1 : f);
          int fz = -1, br = 0;
          if (frozen && s != 0.0)
            fz = (frozen[MIX(i, f)] >> (p == 0 ? 4 : 6)) & 3;
          double wl[NM];
          limit_wave(limiter, w[f + 1][p], w[up + 1][p], fz, wl, &br);
          if (s != 0.0) mask_bits |= br << (p == 0 ? 4 : 6);
          const double coef = 0.5 * fabs(s) * (1.0 - dtdy * fabs(s));
          for (int m = 0; m < NM; ++m) G[f][m] += coef * wl[m];
        }
        if (!interior) continue;
        for (int m = 0; m < NM; ++m) Gc[GC(f, i) + m] = G[f][m];
        /* the x-sweep wrote the low nibble of rows 0..my-1 only; this
         * column's loop is the only writer of the high nibble */
        if (masks_out) {
          if (f < my) {
            /* ordering: x-sweep finished before this parallel loop */
            masks_out[MIX(i, f)] =
                (uint8_t)((masks_out[MIX(i, f)] & 0x0F) | mask_bits);
          } else {
            masks_out[MIX(i, f)] = (uint8_t)mask_bits;
          }
        }
      }
    for (int f = 0; f <= my; ++f) {
      double bp_[NM], bm_[NM], am[NM], ap[NM];
      for (int m = 0; m < NM; ++m) {
        bp_[m] = apdq_y[AY(f, i) + m];
        bm_[m] = amdq_y[AY(f, i) + m];
        if (tcorr) { /* the variant: B+dQ - 2G, B-dQ + 2G */
          bp_[m] -= 2.0 * G[f][m];
          bm_[m] += 2.0 * G[f][m];
        }
      }
      if (f <= my - 1) { /* B+dQ at edge f enters cell (i, f) */
        split(&ex, bp_, am, ap);
        for (int m = 0; m < NM; ++m) {
          Fy_right[FY(f, i) + m] -= 0.5 * dtdy * ap[m];
          Fy_left[FY(f, i) + m] -= 0.5 * dtdy * am[m];
        }
      }
      if (f >= 1) { /* B-dQ at edge f enters cell (i, f-1) */
        split(&ex, bm_, am, ap);
        for (int m = 0; m < NM; ++m) {
          Fy_right[FY(f - 1, i) + m] -= 0.5 * dtdy * ap[m];
          Fy_left[FY(f - 1, i) + m] -= 0.5 * dtdy * am[m];
        }
      }
    }
    free(G);
    free(w);
  }

  if (terms) {
    for (int j = 0; j < my; ++j)
      for (int e = 0; e <= mx; ++e)
        for (int m = 0; m < NM; ++m) {
          const size_t o = ((size_t)j * (size_t)(mx + 1) + (size_t)e) * NM + (size_t)m;
          terms->Fx[o] = Fc[FC(j, e) + m] + Fy_right[FY(j, e - 1) + m] + Fy_left[FY(j, e) + m];
          terms->amx[o] = amdq_x[AX(j, e) + m];
          terms->apx[o] = apdq_x[AX(j, e) + m];
        }
    for (int f = 0; f <= my; ++f)
      for (int i = 0; i < mx; ++i)
        for (int m = 0; m < NM; ++m) {
          const size_t o = ((size_t)f * (size_t)mx + (size_t)i) * NM + (size_t)m;
          terms->Gy[o] = Gc[GC(f, i) + m] + Gx_top[GX(f - 1, i) + m] + Gx_bot[GX(f, i) + m];
          terms->amy[o] = amdq_y[AY(f, i) + m];
          terms->apy[o] = apdq_y[AY(f, i) + m];
        }
  }

  /* ---- update, eq. (2.3) ---- */
  if (q_out != q_in) memcpy(q_out, q_in, sizeof(double) * NM * (size_t)(mx + 4) * (size_t)(my + 4));
#pragma omp parallel for if (par) schedule(static)
  for (int j = 0; j < my; ++j)
    for (int i = 0; i < mx; ++i)
      for (int m = 0; m < NM; ++m) {
        /* F~ at the left (i-1/2) and right (i+1/2) edges of the cell */
        const double FL = Fc[FC(j, i) + m] + Fy_right[FY(j, i - 1) + m] + Fy_left[FY(j, i) + m];
        const double FR = Fc[FC(j, i + 1) + m] + Fy_right[FY(j, i) + m] + Fy_left[FY(j, i + 1) + m];
        /* G~ at the bottom (j-1/2) and top (j+1/2) edges of the cell */
        const double GB = Gc[GC(j, i) + m] + Gx_top[GX(j - 1, i) + m] + Gx_bot[GX(j, i) + m];
        const double GT = Gc[GC(j + 1, i) + m] + Gx_top[GX(j, i) + m] + Gx_bot[GX(j + 1, i) + m];
        const double fluct_x = apdq_x[AX(j, i) + m] + amdq_x[AX(j, i + 1) + m];
        const double fluct_y = apdq_y[AY(j, i) + m] + amdq_y[AY(j + 1, i) + m];
        q_out[QIX(m, i, j)] = q_in[QIX(m, i, j)] - dtdx * fluct_x - dtdy * fluct_y -
                              dtdx * (FR - FL) - dtdy * (GT - GB);
      }

  /* ---- Courant number, eq. (2.10), over the edges of interior cells ---- */
  if (cfl_out) {
    double cfl = 0.0;
    for (int j = 0; j < my; ++j)
      for (int e = 0; e <= mx; ++e)
        for (int p = 0; p < NW; ++p) cfl = fmax(cfl, fabs(ex.s[p]) * dtdx);
    for (int f = 0; f <= my; ++f)
      for (int i = 0; i < mx; ++i)
        for (int p = 0; p < NW; ++p) cfl = fmax(cfl, fabs(ey.s[p]) * dtdy);
    *cfl_out = cfl;
  }

#undef AX
#undef AY
#undef FC
#undef GC
#undef GX
#undef FY
done:
  free(amdq_x); free(apdq_x); free(amdq_y); free(apdq_y);
  free(Fc); free(Gc); free(Gx_top); free(Gx_bot); free(Fy_right); free(Fy_left);
  return rc;
}

int oracle_step_ex(const double *q_in, double *q_out, int mx, int my,
                   double dx, double dy, double dt, double rho, double K,
                   int limiter, int options, const uint8_t *frozen,
                   uint8_t *masks_out, double *cfl_out, int parallel) {
  return step_core(q_in, q_out, mx, my, dx, dy, dt, rho, K, limiter, options, frozen,
                   masks_out, cfl_out, parallel, NULL);
}

/* The edge terms of one step of q_in (layouts as in edge_terms_t); the new
 * state itself is discarded. */
int oracle_step_terms(const double *q_in, int mx, int my, double dx, double dy,
                      double dt, double rho, double K, int limiter, int options,
                      double *Fx, double *amx, double *apx, double *Gy,
                      double *amy, double *apy) {
  if (mx < 1 || my < 1) return -1;
  double *tmp = malloc(sizeof(double) * NM * (size_t)(mx + 4) * (size_t)(my + 4));
  if (!tmp) return -1;
  const edge_terms_t t = {Fx, amx, apx, Gy, amy, apy};
  const int rc = step_core(q_in, tmp, mx, my, dx, dy, dt, rho, K, limiter, options, NULL,
                           NULL, NULL, 1, &t);
  free(tmp);
  return rc;
}

int oracle_step(const double *q_in, double *q_out, int mx, int my, double dx,
                double dy, double dt, double rho, double K, int limiter,
                double *cfl_out) {
  return oracle_step_ex(q_in, q_out, mx, my, dx, dy, dt, rho, K, limiter, 0,
                        NULL, NULL, cfl_out, 1);
}

/* Many independent patches, one OpenMP task per patch.  Patch k lives at
 * q_in + off[k] (doubles), dims mx[k] x my[k]; cfl_out[k] per patch. */
int oracle_step_patches(int n, const double *q_in, double *q_out,
                        const int64_t *off, const int *mx, const int *my,
                        const double *dx, const double *dy, const double *dt,
                        const double *rho, const double *K, int limiter,
                        double *cfl_out) {
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
  for (int k = 0; k < n; ++k) {
    int r = oracle_step_ex(q_in + off[k], q_out + off[k], mx[k], my[k], dx[k],
                           dy[k], dt[k], rho[k], K[k], limiter, 0, NULL, NULL,
                           cfl_out ? &cfl_out[k] : NULL, 0);
    bad |= (r != 0);
  }
  return bad ? -1 : 0;
}

/* ---------------------------------------------------------------------- */
/* One step in a heterogeneous medium (rho, K per cell)                    */
/* ---------------------------------------------------------------------- */
/*
 * The same unsplit step, eq. (2.3), for q_t + A(x,y) q_x + B(x,y) q_y = 0
 * with A, B of Sec. 4.1 eq. (4.2) taken cell by cell (rho, K: padded
 * [my+4][mx+4] like one plane of q; c = sqrt(K/rho), Z = rho c).
 *
 * Normal solve at the edge between cells l and r (x: A; y: B with v): the
 * jump is split into a left-going wave along (-Z_l, 1, 0) with speed -c_l
 * and a right-going wave along (Z_r, 1, 0) with speed +c_r (plus the
 * speed-0 tangential wave), i.e. strengths
 *   a1 = (-dp + Z_r du)/(Z_l + Z_r),  a2 = (dp + Z_l du)/(Z_l + Z_r),
 * A-dQ = -c_l W1, A+dQ = +c_r W2 (the wave decomposition of the jump in the
 * eigenvectors of the two cells).  Limiter as in the constant medium, on the
 * wave vectors (theta = W_upwind . W / W . W).  Transverse solve of a
 * fluctuation a entering cell m: the part going down is the down-going wave
 * of the Riemann problem between the cell below (b) and m,
 *   B-a = -c_b beta (-Z_b, 0, 1), beta = (-a_p + Z_m a_v)/(Z_b + Z_m),
 * the part going up the up-going wave between m and the cell above (t),
 *   B+a = +c_t beta (Z_t, 0, 1), beta = (a_p + Z_m a_v)/(Z_m + Z_t);
 * mirror images in x.  Courant number: max over the edges of interior cells
 * of max(c_l, c_r) dt/dx (x) and max(c_b, c_t) dt/dy (y).
 */
#define VIX(i, j) ((size_t)((j) + 2) * (size_t)(mx + 4) + (size_t)((i) + 2))

/* dir 0: x (normal velocity u = component 1), 1: y (v = component 2) */
static void riemann_var(int dir, double Zl, double cl, double Zr, double cr,
                        const double ql[NM], const double qr[NM], double W[2][NM],
                        double s[2], double am[NM], double ap[NM]) {
  const int n = dir == 0 ? 1 : 2;
  const double dp = qr[0] - ql[0], dn = qr[n] - ql[n];
  const double a1 = (-dp + Zr * dn) / (Zl + Zr);
  const double a2 = (dp + Zl * dn) / (Zl + Zr);
  for (int m = 0; m < NM; ++m) W[0][m] = W[1][m] = 0.0;
  W[0][0] = -Zl * a1;
  W[0][n] = a1;
  W[1][0] = Zr * a2;
  W[1][n] = a2;
  s[0] = -cl;
  s[1] = cr;
  for (int m = 0; m < NM; ++m) {
    am[m] = s[0] * W[0][m];
    ap[m] = s[1] * W[1][m];
  }
}

/* split a (entering cell m) by the other direction's waves: down (left)
 * with the cell below (left) b, up (right) with the cell above (right) t */
static void split_var(int dir, const double a[NM], double Zb, double cb, double Zm,
                      double Zt, double ct, double minus[NM], double plus[NM]) {
  const int n = dir == 0 ? 1 : 2; /* the normal velocity of the split direction */
  const double bd = (-a[0] + Zm * a[n]) / (Zb + Zm);
  const double bu = (a[0] + Zm * a[n]) / (Zm + Zt);
  for (int m = 0; m < NM; ++m) minus[m] = plus[m] = 0.0;
  minus[0] = -cb * bd * (-Zb);
  minus[n] = -cb * bd;
  plus[0] = ct * bu * Zt;
  plus[n] = ct * bu;
}

int oracle_step_var(const double *q_in, double *q_out, int mx, int my, double dx, double dy,
                    double dt, const double *rho, const double *K, int limiter,
                    double *cfl_out) {
  if (mx < 1 || my < 1 || !(dx > 0.0) || !(dy > 0.0) || !rho || !K) return -1;
  const double dtdx = dt / dx, dtdy = dt / dy;
  const size_t np = (size_t)(mx + 4) * (size_t)(my + 4);
  double *Zc = malloc(sizeof(double) * np), *cc = malloc(sizeof(double) * np);
  const size_t nxe = (size_t)(my + 2) * (size_t)(mx + 1);
  const size_t nye = (size_t)(my + 1) * (size_t)(mx + 2);
  double *amdq_x = calloc(nxe * NM, sizeof(double)), *apdq_x = calloc(nxe * NM, sizeof(double));
  double *amdq_y = calloc(nye * NM, sizeof(double)), *apdq_y = calloc(nye * NM, sizeof(double));
  double *Fc = calloc((size_t)my * (mx + 1) * NM, sizeof(double));
  double *Gc = calloc((size_t)(my + 1) * mx * NM, sizeof(double));
  double *Gx_top = calloc((size_t)(my + 2) * mx * NM, sizeof(double));
  double *Gx_bot = calloc((size_t)(my + 2) * mx * NM, sizeof(double));
  double *Fy_right = calloc((size_t)my * (mx + 2) * NM, sizeof(double));
  double *Fy_left = calloc((size_t)my * (mx + 2) * NM, sizeof(double));
  int rc = 0;
  if (!Zc || !cc || !amdq_x || !apdq_x || !amdq_y || !apdq_y || !Fc || !Gc || !Gx_top ||
      !Gx_bot || !Fy_right || !Fy_left) {
    rc = -1;
    goto done;
  }
  for (size_t k = 0; k < np; ++k) {
    if (!(rho[k] > 0.0) || !(K[k] > 0.0)) {
      rc = -1;
      goto done;
    }
    cc[k] = sqrt(K[k] / rho[k]);
    Zc[k] = rho[k] * cc[k];
  }
#define AX(j, e) (((size_t)((j) + 1) * (size_t)(mx + 1) + (size_t)(e)) * NM)
#define AY(f, i) (((size_t)(f) * (size_t)(mx + 2) + (size_t)((i) + 1)) * NM)
#define FC(j, e) (((size_t)(j) * (size_t)(mx + 1) + (size_t)(e)) * NM)
#define GC(f, i) (((size_t)(f) * (size_t)mx + (size_t)(i)) * NM)
#define GX(j, i) (((size_t)((j) + 1) * (size_t)mx + (size_t)(i)) * NM)
#define FY(j, i) (((size_t)(j) * (size_t)(mx + 2) + (size_t)((i) + 1)) * NM)

  /* ---- x-direction: rows j = -1..my ---- */
  for (int j = -1; j <= my; ++j) {
    double(*W)[2][NM] = malloc(sizeof(double[2][NM]) * (size_t)(mx + 3));
    for (int e = -1; e <= mx + 1; ++e) {
      double ql[NM], qr[NM], am[NM], ap[NM], s[2];
      for (int m = 0; m < NM; ++m) {
        ql[m] = q_in[QIX(m, e - 1, j)];
        qr[m] = q_in[QIX(m, e, j)];
      }
      riemann_var(0, Zc[VIX(e - 1, j)], cc[VIX(e - 1, j)], Zc[VIX(e, j)], cc[VIX(e, j)], ql, qr,
                  W[e + 1], s, am, ap);
      if (e >= 0 && e <= mx)
        for (int m = 0; m < NM; ++m) {
          amdq_x[AX(j, e) + m] = am[m];
          apdq_x[AX(j, e) + m] = ap[m];
        }
    }
    if (j >= 0 && j < my)
      for (int e = 0; e <= mx; ++e) {
        const double sp[2] = {-cc[VIX(e - 1, j)], cc[VIX(e, j)]};
        for (int p = 0; p < 2; ++p) {
          const int up = p == 0 ? e + 1 : e - 1; /* wave 0 goes left, wave 1 right */
          double wl[NM];
          limit_wave(limiter, W[e + 1][p], W[up + 1][p], -1, wl, NULL);
          const double coef = 0.5 * fabs(sp[p]) * (1.0 - dtdx * fabs(sp[p]));
          for (int m = 0; m < NM; ++m) Fc[FC(j, e) + m] += coef * wl[m];
        }
      }
    /* transverse: A+dQ at edge e enters cell e, A-dQ enters cell e-1 */
    for (int e = 0; e <= mx; ++e) {
      double bm[NM], bp[NM];
      if (e <= mx - 1) {
        split_var(1, &apdq_x[AX(j, e)], Zc[VIX(e, j - 1)], cc[VIX(e, j - 1)], Zc[VIX(e, j)],
                  Zc[VIX(e, j + 1)], cc[VIX(e, j + 1)], bm, bp);
        for (int m = 0; m < NM; ++m) {
          Gx_top[GX(j, e) + m] -= 0.5 * dtdx * bp[m];
          Gx_bot[GX(j, e) + m] -= 0.5 * dtdx * bm[m];
        }
      }
      if (e >= 1) {
        split_var(1, &amdq_x[AX(j, e)], Zc[VIX(e - 1, j - 1)], cc[VIX(e - 1, j - 1)],
                  Zc[VIX(e - 1, j)], Zc[VIX(e - 1, j + 1)], cc[VIX(e - 1, j + 1)], bm, bp);
        for (int m = 0; m < NM; ++m) {
          Gx_top[GX(j, e - 1) + m] -= 0.5 * dtdx * bp[m];
          Gx_bot[GX(j, e - 1) + m] -= 0.5 * dtdx * bm[m];
        }
      }
    }
    free(W);
  }

  /* ---- y-direction: columns i = -1..mx ---- */
  for (int i = -1; i <= mx; ++i) {
    double(*W)[2][NM] = malloc(sizeof(double[2][NM]) * (size_t)(my + 3));
    for (int f = -1; f <= my + 1; ++f) {
      double ql[NM], qr[NM], bm[NM], bp[NM], s[2];
      for (int m = 0; m < NM; ++m) {
        ql[m] = q_in[QIX(m, i, f - 1)];
        qr[m] = q_in[QIX(m, i, f)];
      }
      riemann_var(1, Zc[VIX(i, f - 1)], cc[VIX(i, f - 1)], Zc[VIX(i, f)], cc[VIX(i, f)], ql, qr,
                  W[f + 1], s, bm, bp);
      if (f >= 0 && f <= my)
        for (int m = 0; m < NM; ++m) {
          amdq_y[AY(f, i) + m] = bm[m];
          apdq_y[AY(f, i) + m] = bp[m];
        }
    }
    if (i >= 0 && i < mx)
      for (int f = 0; f <= my; ++f) {
        const double sp[2] = {-cc[VIX(i, f - 1)], cc[VIX(i, f)]};
        for (int p = 0; p < 2; ++p) {
          const int up = p == 0 ? f + 1 : f - 1;
          double wl[NM];
          limit_wave(limiter, W[f + 1][p], W[up + 1][p], -1, wl, NULL);
          const double coef = 0.5 * fabs(sp[p]) * (1.0 - dtdy * fabs(sp[p]));
          for (int m = 0; m < NM; ++m) Gc[GC(f, i) + m] += coef * wl[m];
        }
      }
    for (int f = 0; f <= my; ++f) {
      double am[NM], ap[NM];
      if (f <= my - 1) { /* B+dQ at edge f enters cell (i, f) */
        split_var(0, &apdq_y[AY(f, i)], Zc[VIX(i - 1, f)], cc[VIX(i - 1, f)], Zc[VIX(i, f)],
                  Zc[VIX(i + 1, f)], cc[VIX(i + 1, f)], am, ap);
        for (int m = 0; m < NM; ++m) {
          Fy_right[FY(f, i) + m] -= 0.5 * dtdy * ap[m];
          Fy_left[FY(f, i) + m] -= 0.5 * dtdy * am[m];
        }
      }
      if (f >= 1) { /* B-dQ at edge f enters cell (i, f-1) */
        split_var(0, &amdq_y[AY(f, i)], Zc[VIX(i - 1, f - 1)], cc[VIX(i - 1, f - 1)],
                  Zc[VIX(i, f - 1)], Zc[VIX(i + 1, f - 1)], cc[VIX(i + 1, f - 1)], am, ap);
        for (int m = 0; m < NM; ++m) {
          Fy_right[FY(f - 1, i) + m] -= 0.5 * dtdy * ap[m];
          Fy_left[FY(f - 1, i) + m] -= 0.5 * dtdy * am[m];
        }
      }
    }
    free(W);
  }

  /* ---- update, eq. (2.3) ---- */
  if (q_out != q_in) memcpy(q_out, q_in, sizeof(double) * NM * np);
  for (int j = 0; j < my; ++j)
    for (int i = 0; i < mx; ++i)
      for (int m = 0; m < NM; ++m) {
        const double FL = Fc[FC(j, i) + m] + Fy_right[FY(j, i - 1) + m] + Fy_left[FY(j, i) + m];
        const double FR = Fc[FC(j, i + 1) + m] + Fy_right[FY(j, i) + m] + Fy_left[FY(j, i + 1) + m];
        const double GB = Gc[GC(j, i) + m] + Gx_top[GX(j - 1, i) + m] + Gx_bot[GX(j, i) + m];
        const double GT = Gc[GC(j + 1, i) + m] + Gx_top[GX(j, i) + m] + Gx_bot[GX(j + 1, i) + m];
        const double fluct_x = apdq_x[AX(j, i) + m] + amdq_x[AX(j, i + 1) + m];
        const double fluct_y = apdq_y[AY(j, i) + m] + amdq_y[AY(j + 1, i) + m];
        q_out[QIX(m, i, j)] = q_in[QIX(m, i, j)] - dtdx * fluct_x - dtdy * fluct_y -
                              dtdx * (FR - FL) - dtdy * (GT - GB);
      }

  /* ---- Courant number over the edges of interior cells ---- */
  if (cfl_out) {
    double cfl = 0.0;
    for (int j = 0; j < my; ++j)
      for (int e = 0; e <= mx; ++e)
        cfl = fmax(cfl, fmax(cc[VIX(e - 1, j)], cc[VIX(e, j)]) * dtdx);
    for (int f = 0; f <= my; ++f)
      for (int i = 0; i < mx; ++i)
        cfl = fmax(cfl, fmax(cc[VIX(i, f - 1)], cc[VIX(i, f)]) * dtdy);
    *cfl_out = cfl;
  }
#undef AX
#undef AY
#undef FC
#undef GC
#undef GX
#undef FY
done:
  free(Zc); free(cc);
  free(amdq_x); free(apdq_x); free(amdq_y); free(apdq_y);
  free(Fc); free(Gc); free(Gx_top); free(Gx_bot); free(Fy_right); free(Fy_left);
  return rc;
}
#undef VIX

/* ---------------------------------------------------------------------- */
/* Exported single-edge hooks, used by the oracle's own pin tests          */
/* ---------------------------------------------------------------------- */
/* Riemann solve at one edge in direction dir (0: x with A, 1: y with B).
 * waves: 3x3 (wave-major), s: 3 speeds. */
void oracle_riemann_edge(int dir, double rho, double K, const double *ql,
                         const double *qr, double *waves, double *s,
                         double *amdq, double *apdq) {
  eig_t e;
  acoustics_eig(rho, K, dir, &e);
  double w[NW][NM];
  riemann(&e, ql, qr, 0, w, amdq, apdq);
  for (int p = 0; p < NW; ++p) {
    s[p] = e.s[p];
    for (int m = 0; m < NM; ++m) waves[p * NM + m] = w[p][m];
  }
}

/* Transverse split of a vector by direction dir's eigen-structure. */
void oracle_split_vec(int dir, double rho, double K, const double *a,
                      double *minus, double *plus) {
  eig_t e;
  acoustics_eig(rho, K, dir, &e);
  split(&e, a, minus, plus);
}

/* ---------------------------------------------------------------------- */
/* Adjoint of one frozen-branch step, boundary fill included               */
/* ---------------------------------------------------------------------- */
/* With the MC branches frozen (masks recorded by a forward step), one step
 * Q^n -> Q^{n+1} of the interior is the linear map S = U o E: E fills the
 * ghosts from the interior (extrapolation; bc_kind < 0: ghosts are frozen
 * input, E adds nothing), U is the update above.  This applies S^T to a
 * cotangent of the interior of Q^{n+1} by running the forward stages in
 * reverse, each transposed in scatter form: update -> F~/G~ -> transverse
 * splits -> limited corrections and fluctuations -> waves -> jumps -> E^T.
 * lam_next, lam_out: [3][my][mx]. */

/* coefficients (own, upwind) of the frozen limited wave for a branch */
static void frozen_coefs(int b, double *c0, double *c1) {
  switch (b) {
  case 0: *c0 = 0.0; *c1 = 0.0; break;
  case 1: *c0 = 0.5; *c1 = 0.5; break;
  case 2: *c0 = 2.0; *c1 = 0.0; break;
  default: *c0 = 0.0; *c1 = 2.0; break;
  }
}

/* transpose of split(): given cotangents of the minus and plus parts, add
 * Mm^T lm + Mp^T lp to out (M = sum over waves of s r l^T). */
static void split_T(const eig_t *e, const double lm[NM], const double lp[NM], double out[NM]) {
  for (int p = 0; p < NW; ++p) {
    const double *lam = (e->s[p] < 0.0) ? lm : (e->s[p] > 0.0 ? lp : NULL);
    if (!lam) continue;
    double rdot = 0.0;
    for (int m = 0; m < NM; ++m) rdot += e->R[m][p] * lam[m];
    for (int m = 0; m < NM; ++m) out[m] += e->s[p] * rdot * e->L[p][m];
  }
}

int oracle_adjoint_step(const double *lam_next, double *lam_out, int mx, int my, double dx,
                        double dy, double dt, double rho, double K, const uint8_t *masks,
                        int bc_kind) {
  if (mx < 1 || my < 1 || !masks) return -1;
  eig_t ex, ey;
  acoustics_eig(rho, K, 0, &ex);
  acoustics_eig(rho, K, 1, &ey);
  const double dtdx = dt / dx, dtdy = dt / dy;
  const size_t npad = (size_t)(mx + 4) * (size_t)(my + 4);
#define LI(m, i, j) (((size_t)(m) * (size_t)my + (size_t)(j)) * (size_t)mx + (size_t)(i))
#define PI(i, j) ((size_t)((j) + 2) * (size_t)(mx + 4) + (size_t)((i) + 2))
  /* cotangents, laid out like the forward arrays */
  double *lpad = calloc(npad * NM, sizeof(double));                      /* [cell][m] */
  double *l_amdq_x = calloc((size_t)(my + 2) * (mx + 1) * NM, sizeof(double));
  double *l_apdq_x = calloc((size_t)(my + 2) * (mx + 1) * NM, sizeof(double));
  double *l_amdq_y = calloc((size_t)(my + 1) * (mx + 2) * NM, sizeof(double));
  double *l_apdq_y = calloc((size_t)(my + 1) * (mx + 2) * NM, sizeof(double));
  double *l_Ft = calloc((size_t)my * (mx + 1) * NM, sizeof(double));     /* F~ */
  double *l_Gt = calloc((size_t)(my + 1) * mx * NM, sizeof(double));     /* G~ */
  double *l_Gx_top = calloc((size_t)(my + 2) * mx * NM, sizeof(double));
  double *l_Gx_bot = calloc((size_t)(my + 2) * mx * NM, sizeof(double));
  double *l_Fy_right = calloc((size_t)my * (mx + 2) * NM, sizeof(double));
  double *l_Fy_left = calloc((size_t)my * (mx + 2) * NM, sizeof(double));
  /* wave cotangents: x rows -1..my, edges -1..mx+1; y columns -1..mx, edges -1..my+1 */
  double *l_Wx = calloc((size_t)(my + 2) * (mx + 3) * NW * NM, sizeof(double));
  double *l_Wy = calloc((size_t)(mx + 2) * (my + 3) * NW * NM, sizeof(double));
  int rc = 0;
  if (!lpad || !l_amdq_x || !l_apdq_x || !l_amdq_y || !l_apdq_y || !l_Ft || !l_Gt ||
      !l_Gx_top || !l_Gx_bot || !l_Fy_right || !l_Fy_left || !l_Wx || !l_Wy) {
    rc = -1;
    goto done;
  }
#define AX(j, e) (((size_t)((j) + 1) * (size_t)(mx + 1) + (size_t)(e)) * NM)
#define AY(f, i) (((size_t)(f) * (size_t)(mx + 2) + (size_t)((i) + 1)) * NM)
#define FT(j, e) (((size_t)(j) * (size_t)(mx + 1) + (size_t)(e)) * NM)
#define GT(f, i) (((size_t)(f) * (size_t)mx + (size_t)(i)) * NM)
#define GX(j, i) (((size_t)((j) + 1) * (size_t)mx + (size_t)(i)) * NM)
#define FY(j, i) (((size_t)(j) * (size_t)(mx + 2) + (size_t)((i) + 1)) * NM)
#define WX(j, e, p) ((((size_t)((j) + 1) * (size_t)(mx + 3) + (size_t)((e) + 1)) * NW + (p)) * NM)
#define WY(i, f, p) ((((size_t)((i) + 1) * (size_t)(my + 3) + (size_t)((f) + 1)) * NW + (p)) * NM)

  /* ---- update, eq. (2.3), transposed ---- */
  for (int j = 0; j < my; ++j)
    for (int i = 0; i < mx; ++i)
      for (int m = 0; m < NM; ++m) {
        const double l = lam_next[LI(m, i, j)];
        lpad[PI(i, j) * NM + m] += l;
        l_apdq_x[AX(j, i) + m] -= dtdx * l;
        l_amdq_x[AX(j, i + 1) + m] -= dtdx * l;
        l_apdq_y[AY(j, i) + m] -= dtdy * l;
        l_amdq_y[AY(j + 1, i) + m] -= dtdy * l;
        l_Ft[FT(j, i + 1) + m] -= dtdx * l;
        l_Ft[FT(j, i) + m] += dtdx * l;
        l_Gt[GT(j + 1, i) + m] -= dtdy * l;
        l_Gt[GT(j, i) + m] += dtdy * l;
      }
  /* ---- F~ = Fc + transverse parts; G~ likewise ---- */
  for (int j = 0; j < my; ++j)
    for (int e = 0; e <= mx; ++e)
      for (int m = 0; m < NM; ++m) {
        l_Fy_right[FY(j, e - 1) + m] += l_Ft[FT(j, e) + m];
        l_Fy_left[FY(j, e) + m] += l_Ft[FT(j, e) + m];
      }
  for (int f = 0; f <= my; ++f)
    for (int i = 0; i < mx; ++i)
      for (int m = 0; m < NM; ++m) {
        l_Gx_top[GX(f - 1, i) + m] += l_Gt[GT(f, i) + m];
        l_Gx_bot[GX(f, i) + m] += l_Gt[GT(f, i) + m];
      }
  /* ---- transverse splits, transposed ---- */
  for (int j = -1; j <= my; ++j)
    for (int e = 0; e <= mx; ++e) {
      double acc[NM] = {0, 0, 0}, lm[NM], lp[NM];
      if (e <= mx - 1) { /* A+dQ at edge e entered cell e */
        for (int m = 0; m < NM; ++m) {
          lm[m] = -0.5 * dtdx * l_Gx_bot[GX(j, e) + m];
          lp[m] = -0.5 * dtdx * l_Gx_top[GX(j, e) + m];
        }
        split_T(&ey, lm, lp, acc);
        for (int m = 0; m < NM; ++m) l_apdq_x[AX(j, e) + m] += acc[m];
      }
      if (e >= 1) { /* A-dQ at edge e entered cell e-1 */
        for (int m = 0; m < NM; ++m) {
          acc[m] = 0.0;
          lm[m] = -0.5 * dtdx * l_Gx_bot[GX(j, e - 1) + m];
          lp[m] = -0.5 * dtdx * l_Gx_top[GX(j, e - 1) + m];
        }
        split_T(&ey, lm, lp, acc);
        for (int m = 0; m < NM; ++m) l_amdq_x[AX(j, e) + m] += acc[m];
      }
    }
  for (int i = -1; i <= mx; ++i)
    for (int f = 0; f <= my; ++f) {
      double acc[NM] = {0, 0, 0}, lm[NM], lp[NM];
      if (f <= my - 1) {
        for (int m = 0; m < NM; ++m) {
          lm[m] = -0.5 * dtdy * l_Fy_left[FY(f, i) + m];
          lp[m] = -0.5 * dtdy * l_Fy_right[FY(f, i) + m];
        }
        split_T(&ex, lm, lp, acc);
        for (int m = 0; m < NM; ++m) l_apdq_y[AY(f, i) + m] += acc[m];
      }
      if (f >= 1) {
        for (int m = 0; m < NM; ++m) {
          acc[m] = 0.0;
          lm[m] = -0.5 * dtdy * l_Fy_left[FY(f - 1, i) + m];
          lp[m] = -0.5 * dtdy * l_Fy_right[FY(f - 1, i) + m];
        }
        split_T(&ex, lm, lp, acc);
        for (int m = 0; m < NM; ++m) l_amdq_y[AY(f, i) + m] += acc[m];
      }
    }
  /* ---- limited corrections (frozen branches) and fluctuations -> waves ---- */
  for (int j = 0; j < my; ++j)
    for (int e = 0; e <= mx; ++e)
      for (int p = 0; p < NW; ++p) {
        const double s = ex.s[p];
        if (s == 0.0) continue;
        const int up = (s > 0.0) ? e - 1 : e + 1;
        const int b = (masks[MIX(e, j)] >> (p == 0 ? 0 : 2)) & 3;
        double c0, c1;
        frozen_coefs(b, &c0, &c1);
        const double coef = 0.5 * fabs(s) * (1.0 - dtdx * fabs(s));
        for (int m = 0; m < NM; ++m) {
          l_Wx[WX(j, e, p) + m] += coef * c0 * l_Ft[FT(j, e) + m];
          l_Wx[WX(j, up, p) + m] += coef * c1 * l_Ft[FT(j, e) + m];
        }
      }
  for (int i = 0; i < mx; ++i)
    for (int f = 0; f <= my; ++f)
      for (int p = 0; p < NW; ++p) {
        const double s = ey.s[p];
        if (s == 0.0) continue;
        const int up = (s > 0.0) ? f - 1 : f + 1;
        const int b = (masks[MIX(i, f)] >> (p == 0 ? 4 : 6)) & 3;
        double c0, c1;
        frozen_coefs(b, &c0, &c1);
        const double coef = 0.5 * fabs(s) * (1.0 - dtdy * fabs(s));
        for (int m = 0; m < NM; ++m) {
          l_Wy[WY(i, f, p) + m] += coef * c0 * l_Gt[GT(f, i) + m];
          l_Wy[WY(i, up, p) + m] += coef * c1 * l_Gt[GT(f, i) + m];
        }
      }
  for (int j = -1; j <= my; ++j)
    for (int e = 0; e <= mx; ++e)
      for (int p = 0; p < NW; ++p) {
        const double s = ex.s[p];
        for (int m = 0; m < NM; ++m) {
          if (s < 0.0) l_Wx[WX(j, e, p) + m] += s * l_amdq_x[AX(j, e) + m];
          else if (s > 0.0) l_Wx[WX(j, e, p) + m] += s * l_apdq_x[AX(j, e) + m];
        }
      }
  for (int i = -1; i <= mx; ++i)
    for (int f = 0; f <= my; ++f)
      for (int p = 0; p < NW; ++p) {
        const double s = ey.s[p];
        for (int m = 0; m < NM; ++m) {
          if (s < 0.0) l_Wy[WY(i, f, p) + m] += s * l_amdq_y[AY(f, i) + m];
          else if (s > 0.0) l_Wy[WY(i, f, p) + m] += s * l_apdq_y[AY(f, i) + m];
        }
      }
  /* ---- waves W = alpha r, alpha = L (q_r - q_l) -> cell cotangents ---- */
  for (int j = -1; j <= my; ++j)
    for (int e = -1; e <= mx + 1; ++e) {
      double ldq[NM] = {0, 0, 0};
      for (int p = 0; p < NW; ++p) {
        double la = 0.0;
        for (int m = 0; m < NM; ++m) la += ex.R[m][p] * l_Wx[WX(j, e, p) + m];
        for (int m = 0; m < NM; ++m) ldq[m] += la * ex.L[p][m];
      }
      for (int m = 0; m < NM; ++m) {
        lpad[PI(e, j) * NM + m] += ldq[m];
        lpad[PI(e - 1, j) * NM + m] -= ldq[m];
      }
    }
  for (int i = -1; i <= mx; ++i)
    for (int f = -1; f <= my + 1; ++f) {
      double ldq[NM] = {0, 0, 0};
      for (int p = 0; p < NW; ++p) {
        double la = 0.0;
        for (int m = 0; m < NM; ++m) la += ey.R[m][p] * l_Wy[WY(i, f, p) + m];
        for (int m = 0; m < NM; ++m) ldq[m] += la * ey.L[p][m];
      }
      for (int m = 0; m < NM; ++m) {
        lpad[PI(i, f) * NM + m] += ldq[m];
        lpad[PI(i, f - 1) * NM + m] -= ldq[m];
      }
    }
  /* ---- boundary fill transposed: E = (y-ghosts over the full width) o
   * (x-ghosts of interior rows), so E^T folds the ghost rows first, then the
   * ghost columns of the interior rows, into the nearest interior cells ---- */
  if (bc_kind == OR_BC_EXTRAP) {
    for (int i = -2; i < mx + 2; ++i)
      for (int g = 1; g <= 2; ++g)
        for (int m = 0; m < NM; ++m) {
          lpad[PI(i, 0) * NM + m] += lpad[PI(i, -g) * NM + m];
          lpad[PI(i, my - 1) * NM + m] += lpad[PI(i, my - 1 + g) * NM + m];
        }
    for (int j = 0; j < my; ++j)
      for (int g = 1; g <= 2; ++g)
        for (int m = 0; m < NM; ++m) {
          lpad[PI(0, j) * NM + m] += lpad[PI(-g, j) * NM + m];
          lpad[PI(mx - 1, j) * NM + m] += lpad[PI(mx - 1 + g, j) * NM + m];
        }
  }
  for (int m = 0; m < NM; ++m)
    for (int j = 0; j < my; ++j)
      for (int i = 0; i < mx; ++i) lam_out[LI(m, i, j)] = lpad[PI(i, j) * NM + m];

#undef AX
#undef AY
#undef FT
#undef GT
#undef GX
#undef FY
#undef WX
#undef WY
#undef LI
#undef PI
done:
  free(lpad); free(l_amdq_x); free(l_apdq_x); free(l_amdq_y); free(l_apdq_y);
  free(l_Ft); free(l_Gt); free(l_Gx_top); free(l_Gx_bot); free(l_Fy_right); free(l_Fy_left);
  free(l_Wx); free(l_Wy);
  return rc;
}
