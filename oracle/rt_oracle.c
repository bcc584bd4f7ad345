/*
 * Plain FP64 CPU oracle of the radiative-transfer step of Jiang, Stone &
 * Davis (2014).  TEST INFRASTRUCTURE ONLY: see rt_oracle.h.  Every function
 * follows the paper's Section 4 in the paper's order and notation; nothing is
 * blocked, fused or reordered for speed.  Readings of passages the paper
 * leaves open are stated where they are used.
 */
#include "rt_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define FOURPI (4.0 * M_PI)

int or_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void or_set_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

static long long ncell_of(const or_problem *p) {
  return (long long)p->n[0] * p->n[1] * p->n[2];
}

static long long cidx(const or_problem *p, int x, int y, int z) {
  return (long long)x + (long long)p->n[0] * ((long long)y + (long long)p->n[1] * z);
}

/* ---------------------------------------------------------------- moments */
/* Section 3: the discrete moments J = sum I W, H_i = sum mu_i I W,
 * K_ij = sum mu_i mu_j I W; E_r = 4 pi J, F_r = 4 pi H, P_r = 4 pi K
 * (Section 2, with F_r in units of c a_r T0^4). */
void or_moments(const or_problem *p, const double *I, double *E, double *F,
                double *Pr) {
  const long long nc = ncell_of(p);
  const int N = p->nang;
#pragma omp parallel for schedule(static)
  for (long long c = 0; c < nc; ++c) {
    double J = 0, H[3] = {0, 0, 0}, K[6] = {0, 0, 0, 0, 0, 0};
    for (int m = 0; m < N; ++m) {
      const double *n = p->mu + 3 * m;
      const double Iw = I[(long long)m * nc + c] * p->w[m];
      J += Iw;
      H[0] += n[0] * Iw;
      H[1] += n[1] * Iw;
      H[2] += n[2] * Iw;
      K[0] += n[0] * n[0] * Iw;
      K[1] += n[1] * n[1] * Iw;
      K[2] += n[2] * n[2] * Iw;
      K[3] += n[0] * n[1] * Iw;
      K[4] += n[0] * n[2] * Iw;
      K[5] += n[1] * n[2] * Iw;
    }
    if (E) E[c] = FOURPI * J;
    if (F)
      for (int k = 0; k < 3; ++k) F[(long long)k * nc + c] = FOURPI * H[k];
    if (Pr)
      for (int k = 0; k < 6; ++k) Pr[(long long)k * nc + c] = FOURPI * K[k];
  }
}

/* ------------------------------------------------------------- boundaries */
/* Index of the cell that supplies field values (J, v, sigma) at coordinate k
 * along axis d: periodic wrap, otherwise the last active cell (zero-gradient
 * ghost fields). */
static int field_coord(const or_problem *p, int d, int k) {
  const int n = p->n[d];
  if (k >= 0 && k < n) return k;
  if ((k < 0 && p->bc[d][0] == OR_BC_PERIODIC) ||
      (k >= n && p->bc[d][1] == OR_BC_PERIODIC))
    return ((k % n) + n) % n;
  return k < 0 ? 0 : n - 1;
}

typedef struct {
  const or_problem *p;
  const double *I, *J, *v;
  long long nc;
  int m;          /* angle                                   */
  int d;          /* axis                                    */
  int base[3];    /* coordinates of the line (axis d varies) */
} line_ctx;

static long long line_cell(const line_ctx *L, int k) {
  int q[3] = {L->base[0], L->base[1], L->base[2]};
  q[L->d] = field_coord(L->p, L->d, k);
  return cidx(L->p, q[0], q[1], q[2]);
}

/* Intensity of angle m at coordinate k of the line, with the ghost zones of
 * each boundary kind: periodic wrap; fixed table (beams, inflow); copy of the
 * last active zone for every angle; vacuum = outgoing angles copied and
 * incoming ones zero (Sections 5.3, 5.7, 5.8). */
static double line_I(const line_ctx *L, int k) {
  const or_problem *p = L->p;
  const int n = p->n[L->d];
  if (k >= 0 && k < n) return L->I[(long long)L->m * L->nc + line_cell(L, k)];
  const int side = k < 0 ? 0 : 1;
  const int bc = p->bc[L->d][side];
  if (bc == OR_BC_PERIODIC) return L->I[(long long)L->m * L->nc + line_cell(L, k)];
  if (bc == OR_BC_FIXED) {
    const double *f = p->ghost_face[L->d][side];
    if (!f) return p->ghost[L->d][side][L->m];
    /* the face cell of the line: its coordinates on the two other axes */
    const int a = L->d == 0 ? 1 : 0, b = L->d == 2 ? 1 : 2;
    const long long nface = (long long)p->n[a] * p->n[b];
    return f[(long long)L->m * nface + L->base[a] + (long long)p->n[a] * L->base[b]];
  }
  const double mu = p->mu[3 * L->m + L->d];
  const int outgoing = side == 0 ? (mu < 0) : (mu > 0);
  if (bc == OR_BC_VACUUM && !outgoing) return 0.0;
  return L->I[(long long)L->m * L->nc + line_cell(L, k)];
}

/* IV = 3 n.v J (Section 4.2), the velocity-dependent part of the intensity. */
static double line_IV(const line_ctx *L, int k) {
  if (L->p->original) return 0.0; /* no IV split: I~ = I, no IV flux */
  const long long c = line_cell(L, k);
  const double *n = L->p->mu + 3 * L->m;
  const double nv = n[0] * L->v[c] + n[1] * L->v[L->nc + c] + n[2] * L->v[2 * L->nc + c];
  return 3.0 * nv * L->J[c];
}

/* I~ = I - IV/C (Section 4.2, Eq. transporttwoterms). */
static double line_It(const line_ctx *L, int k) {
  return line_I(L, k) - line_IV(L, k) / L->p->C;
}

/* van Leer (1977) monotonic slope: harmonic mean of the one-sided
 * differences when they share a sign, zero at extrema.  Reading of the
 * second-order scheme the transport flux cites from Stone & Mihalas (1992). */
static double van_leer(double a, double b) {
  const double ab = a * b;
  return ab > 0.0 ? 2.0 * ab / (a + b) : 0.0;
}

/* Upwind interpolated interface value of a piecewise-linear monotonic
 * reconstruction advected at Courant number nu: up1 is the upwind cell,
 * up2 the cell behind it, dn1 the downwind cell. */
static double upwind_face(double up2, double up1, double dn1, double nu) {
  return up1 + 0.5 * (1.0 - nu) * van_leer(up1 - up2, dn1 - up1);
}

/* Reduced transport speed factor alpha = sqrt((1 - exp(-tau))/tau),
 * tau = [10 dl (sigma_a + sigma_s)]^2 (Section 4.2), evaluated at an
 * interface with the mean opacity of its two cells; alpha(0) = 1. */
static double alpha_of(double sigma, double dl) {
  const double s = 10.0 * dl * sigma;
  const double tau = s * s;
  if (tau <= 0.0) return 1.0;
  return sqrt(-expm1(-tau) / tau);
}

/* Flux through the interface between line coordinates k-1 and k:
 *   Phi = C mu [alpha I~*_up + (1 - alpha) I~_c] + mu IV*,
 * where I~*_up is the van Leer upwind value for the direction of mu at
 * Courant number C|mu|dt/dx, I~_c the centred average (the upwind
 * dissipation is scaled by alpha, i.e. a transport speed alpha C), and IV*
 * the van Leer upwind value of IV for the direction of the interface flow
 * speed at Courant number |v|dt/dx (centred when that speed is zero). */
static double face_flux(const line_ctx *L, int k, double dt, const double *sa,
                        const double *ss) {
  const or_problem *p = L->p;
  const int d = L->d;
  const double mu = p->mu[3 * L->m + d];
  const double dl = p->dx[d];
  const long long cL = line_cell(L, k - 1), cR = line_cell(L, k);
  /* Ghost opacities copy the edge cell. */
  const double sig = 0.5 * ((sa[cL] + ss[cL]) + (sa[cR] + ss[cR]));
  const double alpha = L->p->original ? 1.0 : alpha_of(sig, dl);

  double phi_t = 0.0;
  if (mu != 0.0) {
    const double nu = p->C * fabs(mu) * dt / dl;
    double up;
    if (mu > 0)
      up = upwind_face(line_It(L, k - 2), line_It(L, k - 1), line_It(L, k), nu);
    else
      up = upwind_face(line_It(L, k + 1), line_It(L, k), line_It(L, k - 1), nu);
    const double cen = 0.5 * (line_It(L, k - 1) + line_It(L, k));
    phi_t = p->C * mu * (alpha * up + (1.0 - alpha) * cen);
  }

  const double uf = 0.5 * (L->v[(long long)d * L->nc + cL] + L->v[(long long)d * L->nc + cR]);
  double iv;
  if (uf > 0) {
    iv = upwind_face(line_IV(L, k - 2), line_IV(L, k - 1), line_IV(L, k), fabs(uf) * dt / dl);
  } else if (uf < 0) {
    iv = upwind_face(line_IV(L, k + 1), line_IV(L, k), line_IV(L, k - 1), fabs(uf) * dt / dl);
  } else {
    iv = 0.5 * (line_IV(L, k - 1) + line_IV(L, k));
  }
  return phi_t + mu * iv;
}

/* Delta F of one cell and angle: the divergence of the interface fluxes
 * along every active axis, all evaluated from time-n data (unsplit). */
static double cell_dF(const or_problem *p, double dt, const double *I,
                      const double *J, const double *v, const double *sa,
                      const double *ss, int m, int x, int y, int z) {
  const int q[3] = {x, y, z};
  double dF = 0.0;
  for (int d = 0; d < p->ndim; ++d) {
    line_ctx L = {p, I, J, v, ncell_of(p), m, d, {x, y, z}};
    const int k = q[d];
    const double fr = face_flux(&L, k + 1, dt, sa, ss);
    const double fl = face_flux(&L, k, dt, sa, ss);
    dF -= dt * (fr - fl) / p->dx[d];
  }
  return dF;
}

double or_radiation_dt(const or_problem *p, double dt) {
  return p->chat > 0.0 ? dt * (p->chat / p->C) : dt;
}

void or_transport(const or_problem *p, double dt_gas, const double *I,
                  const double *J, const double *v, const double *sa,
                  const double *ss, double *dF) {
  const long long nc = ncell_of(p);
  /* the transport is the radiation's: it advances at the (reduced) speed */
  const double dt = or_radiation_dt(p, dt_gas);
#pragma omp parallel for schedule(static) collapse(2)
  for (int m = 0; m < p->nang; ++m)
    for (int z = 0; z < p->n[2]; ++z)
      for (int y = 0; y < p->n[1]; ++y)
        for (int x = 0; x < p->n[0]; ++x)
          dF[(long long)m * nc + cidx(p, x, y, z)] =
              cell_dF(p, dt, I, J, v, sa, ss, m, x, y, z);
}

/* ----------------------------------------------------- velocity estimate */
/* Section 4.5: solve, per component k,
 *   rho vt - rho v = (dt/2) P sigma [ (C/P) rho v + F - (C/P) rho vt
 *                                      - vt (E + P_kk) / C ]
 * with sigma = sigma_a + sigma_s, holding E and the diagonal P_kk fixed. */
static void vtilde_cell(const or_problem *p, double dt, double rho, double sig,
                        const double *v, const double *F, double E,
                        const double *Pdiag, double *vt) {
  for (int k = 0; k < 3; ++k) {
    if (!p->estimate_v) {
      vt[k] = v[k];
      continue;
    }
    /* multiplied out so that P = 0 is allowed: (dt/2) P sigma (C/P) = (dt/2) sigma C */
    const double h = 0.5 * dt * sig;
    const double num = rho * v[k] + h * (p->C * rho * v[k] + p->P * F[k]);
    const double den = rho + h * (p->C * rho + p->P * (E + Pdiag[k]) / p->C);
    vt[k] = num / den;
  }
}

void or_vtilde(const or_problem *p, double dt, const double *rho,
               const double *sa, const double *ss, const double *v,
               const double *E, const double *F, const double *Pr,
               double *vt) {
  const long long nc = ncell_of(p);
  for (long long c = 0; c < nc; ++c) {
    const double vc[3] = {v[c], v[nc + c], v[2 * nc + c]};
    const double Fc[3] = {F[c], F[nc + c], F[2 * nc + c]};
    const double Pd[3] = {Pr[c], Pr[nc + c], Pr[2 * nc + c]};
    double out[3];
    vtilde_cell(p, dt, rho[c], sa[c] + ss[c], vc, Fc, E[c], Pd, out);
    for (int k = 0; k < 3; ++k) vt[(long long)k * nc + c] = out[k];
  }
}

/* ------------------------------------------------------------ absorption */
/* Section 4.3, Eq. absorptionmatrix: N + 1 equations in I_m^{n+1} and
 * T^{n+1} (velocity u and sigma_a fixed), solved by Newton-Raphson from the
 * initial guess (r, T^n).  The residuals are the equations written as
 * G = lhs - rhs:
 *   G_m = I_m - r_m - dt [ C sa (T^4/4pi - I_m) + 3 (n_m.u) sa T^4/4pi
 *           + (n_m.u) sa I_m - sa (u.u)/C sum_l W_l I_l
 *           - (sa/C) sum_l (u.n_l)^2 W_l I_l ],
 *   G_T = c_v (T - T^n) - dt [ -8pi P sa u.( sum_l n_l W_l I_l
 *           - (1/C) sum_l (u + (u.n_l) n_l) W_l I_l )
 *           - P C (1 - u.u/C^2) sa (T^4 - 4pi sum_l W_l I_l) ],
 * with c_v = rho R_ideal/(gamma - 1).  The Jacobian is inverted as the paper
 * describes: subtracting the row of I_N from every other row of I_m leaves
 * each I_m a function of I_N and T, so only a 2 x 2 system in (dI_N, dT) is
 * solved per iteration (cost O(N)). */
int or_absorption_cell(const or_problem *p, double dt, double sa, double rho,
                       const double *u, const double *r, double Tn,
                       double *Iout, double *Tout) {
  const int N = p->nang;
  /* the rows of the intensities advance by the radiation's time step, the
   * row of the gas temperature by dt (the same unless the speed of light
   * is reduced) */
  const double dtr = or_radiation_dt(p, dt);
  const double C = p->C, P = p->P;
  const double cv = rho * p->R / (p->gamma - 1.0);
  const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  double *I = Iout;
  double *t = (double *)malloc(sizeof(double) * N);     /* n_m . u        */
  double *G = (double *)malloc(sizeof(double) * N);     /* residuals      */
  double *dIa = (double *)malloc(sizeof(double) * N);   /* dI_m coeff dI_N */
  double *dIb = (double *)malloc(sizeof(double) * N);   /* dI_m coeff dT   */
  double *dIc = (double *)malloc(sizeof(double) * N);   /* dI_m constant   */
  for (int m = 0; m < N; ++m) {
    const double *n = p->mu + 3 * m;
    t[m] = n[0] * u[0] + n[1] * u[1] + n[2] * u[2];
    I[m] = r[m];
  }
  double T = Tn;
  int it, converged = 0;
  for (it = 1; it <= p->maxit; ++it) {
    /* sums over angles of the current iterate */
    double sJ = 0, sH = 0, sK = 0;   /* sum W I, sum (u.n) W I, sum (u.n)^2 W I */
    for (int l = 0; l < N; ++l) {
      sJ += p->w[l] * I[l];
      sH += t[l] * p->w[l] * I[l];
      sK += t[l] * t[l] * p->w[l] * I[l];
    }
    const double T4pi = T * T * T * T / FOURPI;
    for (int m = 0; m < N; ++m) {
      const double rhs = C * sa * (T4pi - I[m]) + 3.0 * t[m] * sa * T4pi + t[m] * sa * I[m] -
                         sa * uu / C * sJ - sa / C * sK;
      G[m] = I[m] - r[m] - dtr * rhs;
    }
    const double rhsT = -8.0 * M_PI * P * sa * (sH - (uu * sJ + sK) / C) -
                        P * C * (1.0 - uu / (C * C)) * sa * (T * T * T * T - FOURPI * sJ);
    const double GT = cv * (T - Tn) - dt * rhsT;

    /* Jacobian entries (dtr the radiation's step, dt the gas's):
     *   dG_m/dI_l = delta_ml D_m + kappa g_l W_l,
     *     D_m = 1 + dtr sa (C - t_m), kappa = dtr sa / C, g_l = u.u + t_l^2
     *   dG_m/dT   = -e_m T^3/pi,  e_m = dtr sa (C + 3 t_m)
     *   dG_T/dI_l = gT_l = dt [8pi P sa (t_l - g_l/C) - 4pi P C (1-u.u/C^2) sa] W_l
     *   dG_T/dT   = c_v + 4 dt P C (1 - u.u/C^2) sa T^3 */
    const double kap = dtr * sa / C;
    const double T3pi = T * T * T / M_PI;
    const int Nn = N - 1;
    const double DN = 1.0 + dtr * sa * (C - t[Nn]);
    const double eN = dtr * sa * (C + 3.0 * t[Nn]);
    /* rows m != N minus row N:
     *   D_m dI_m - D_N dI_N - (e_m - e_N) T^3/pi dT = -(G_m - G_N) */
    for (int m = 0; m < N; ++m) {
      if (m == Nn) {
        dIa[m] = 1.0;
        dIb[m] = 0.0;
        dIc[m] = 0.0;
        continue;
      }
      const double Dm = 1.0 + dtr * sa * (C - t[m]);
      const double em = dtr * sa * (C + 3.0 * t[m]);
      dIa[m] = DN / Dm;
      dIb[m] = (em - eN) * T3pi / Dm;
      dIc[m] = -(G[m] - G[Nn]) / Dm;
    }
    /* row N and row T in the unknowns (dI_N, dT) */
    double a11 = DN, a12 = -eN * T3pi, b1 = -G[Nn];
    double a21 = 0.0, a22 = cv + 4.0 * dt * P * C * (1.0 - uu / (C * C)) * sa * T * T * T,
           b2 = -GT;
    for (int l = 0; l < N; ++l) {
      const double gl = uu + t[l] * t[l];
      const double kg = kap * gl * p->w[l];
      const double gT = dt * (8.0 * M_PI * P * sa * (t[l] - gl / C) -
                              FOURPI * P * C * (1.0 - uu / (C * C)) * sa) * p->w[l];
      a11 += kg * dIa[l];
      a12 += kg * dIb[l];
      b1 -= kg * dIc[l];
      a21 += gT * dIa[l];
      a22 += gT * dIb[l];
      b2 -= gT * dIc[l];
    }
    const double det = a11 * a22 - a12 * a21;
    const double dIN = (b1 * a22 - a12 * b2) / det;
    const double dT = (a11 * b2 - a21 * b1) / det;
    double dImax = 0.0, Imax = 0.0;
    for (int m = 0; m < N; ++m) {
      const double dI = dIa[m] * dIN + dIb[m] * dT + dIc[m];
      I[m] += dI;
      if (fabs(dI) > dImax) dImax = fabs(dI);
      if (fabs(I[m]) > Imax) Imax = fabs(I[m]);
    }
    T += dT;
    if (fabs(dT) <= p->rtol * fabs(T) && dImax <= p->rtol * (Imax > 0 ? Imax : 1.0)) {
      converged = 1;
      break;
    }
  }
  *Tout = T;
  free(t);
  free(G);
  free(dIa);
  free(dIb);
  free(dIc);
  if (!converged || !(T > 0.0)) return -1;
  return it;
}

/* ------------------------------------------------------------ scattering */
/* Section 4.4: backward-Euler scattering step with unknowns y_m = I_m W_m,
 * M_s y = r with M_ml = a_m delta_ml + b_l + c_m and
 *   a_m = (1 + dt C ss - dt ss n_m.u) / W_m,
 *   b_m = -dt C ss + 2 dt ss u.n_m - dt ss u.u/C - dt (ss/C) (u.n_m)^2,
 *   c_m = -3 dt ss n_m.u.
 * Solved here by plain Gaussian elimination with partial pivoting of the
 * dense matrix (the paper's analytic LU reaches the same solution). */
int or_scattering_cell(const or_problem *p, double dt_gas, double ss,
                       const double *u, const double *r, double *Iout) {
  const int N = p->nang;
  const double dt = or_radiation_dt(p, dt_gas); /* a radiation-only step */
  if (ss == 0.0) {
    /* no scattering: M_s = diag(1/W_m), so I'_m = r_m */
    for (int m = 0; m < N; ++m) Iout[m] = r[m];
    return 0;
  }
  const double C = p->C;
  const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  double *A = (double *)malloc(sizeof(double) * N * N);
  double *y = (double *)malloc(sizeof(double) * N);
  double *a = (double *)malloc(sizeof(double) * N);
  double *b = (double *)malloc(sizeof(double) * N);
  double *c = (double *)malloc(sizeof(double) * N);
  for (int m = 0; m < N; ++m) {
    const double *n = p->mu + 3 * m;
    const double t = n[0] * u[0] + n[1] * u[1] + n[2] * u[2];
    a[m] = (1.0 + dt * C * ss - dt * ss * t) / p->w[m];
    b[m] = -dt * C * ss + 2.0 * dt * ss * t - dt * ss * uu / C - dt * ss / C * t * t;
    c[m] = -3.0 * dt * t * ss;
  }
  for (int m = 0; m < N; ++m) {
    for (int l = 0; l < N; ++l) A[m * N + l] = b[l] + c[m] + (m == l ? a[m] : 0.0);
    y[m] = r[m];
  }
  int status = 0;
  for (int k = 0; k < N; ++k) {
    int piv = k;
    for (int i = k + 1; i < N; ++i)
      if (fabs(A[i * N + k]) > fabs(A[piv * N + k])) piv = i;
    if (A[piv * N + k] == 0.0) {
      status = -1;
      break;
    }
    if (piv != k) {
      for (int j = 0; j < N; ++j) {
        const double tmp = A[k * N + j];
        A[k * N + j] = A[piv * N + j];
        A[piv * N + j] = tmp;
      }
      const double tmp = y[k];
      y[k] = y[piv];
      y[piv] = tmp;
    }
    for (int i = k + 1; i < N; ++i) {
      const double f = A[i * N + k] / A[k * N + k];
      for (int j = k; j < N; ++j) A[i * N + j] -= f * A[k * N + j];
      y[i] -= f * y[k];
    }
  }
  if (status == 0) {
    for (int k = N - 1; k >= 0; --k) {
      double s = y[k];
      for (int j = k + 1; j < N; ++j) s -= A[k * N + j] * y[j];
      y[k] = s / A[k * N + k];
    }
    for (int m = 0; m < N; ++m) Iout[m] = y[m] / p->w[m];
  }
  free(A);
  free(y);
  free(a);
  free(b);
  free(c);
  return status;
}

/* ----------------------------------------------------------------- step */
/* Source part of one step for one cell (Steps 3-5 and the gas source terms
 * of Step 7), given I^n and Delta F of the cell.
 *   Step 2 routing: Delta F joins the right-hand side of Step 5 when
 *     sigma_s > sigma_a, else of Step 4 (ties, including sigma = 0, go to 4).
 *   Step 4 momentum change: -(4pi P/C) [sum n W I' - sum n W r4], r4 being
 *     the right-hand side of that sub-step (I^n plus Delta F if routed
 *     there); the 4pi converts H to F_r so that rho v + P F_r/C is
 *     conserved.  Step 5 likewise with r5.
 *   Gas internal energy change c_v (T' - T^n), c_v = rho R/(gamma - 1).
 *   Kinetic energy change ((rho v^n + d(rho v))^2 - (rho v^n)^2)/(2 rho).
 * Second order in time (Section 4.3 attributes the O(dt^2) gap between the
 * gas energy change and the radiation energy change to the first-order
 * solve, and names solving the absorption system twice as the cure).
 * Reading: the gap is the work term, which the system takes at the velocity
 * u of the step while the kinetic energy change equals the momentum change
 * times the mean of v^n and v^n + d(rho v)/rho.  So the system is solved a
 * first time at u (the Step 3 estimate, or v^n), giving the Step 4 momentum
 * change d4; then again, from the same right-hand side r4 and T^n, at the
 * time-centred velocity v^n + d4/(2 rho).  The second solution is the
 * step's.  The scattering step keeps u. */
static int source_cell(const or_problem *p, double dt, double rho, double sa,
                       double ss, const double *v, const double *vt,
                       const double *In, const double *dFc, double Tn,
                       double *Inew, double *Tnew, double *dEgas, double *dEkin,
                       double *dMom, double *scratch) {
  const int N = p->nang;
  double *r4 = scratch, *I4 = scratch + N, *r5 = scratch + 2 * N;
  const int to5 = ss > sa;
  for (int m = 0; m < N; ++m) r4[m] = In[m] + (to5 ? 0.0 : dFc[m]);
  double T4;
  /* the gas gains the momentum the radiation loses, at the true rate: C/chat
   * times the radiation's change with a reduced speed of light */
  const double gas = p->chat > 0.0 ? p->C / p->chat : 1.0;
  int it = or_absorption_cell(p, dt, sa, rho, vt, r4, Tn, I4, &T4);
  if (p->second_order && it > 0) {
    double uc[3];
    for (int k = 0; k < 3; ++k) {
      double dH = 0.0; /* sum_m n_m W_m (I'_m - r4_m) */
      for (int m = 0; m < N; ++m) dH += p->mu[3 * m + k] * p->w[m] * (I4[m] - r4[m]);
      const double d4 = -gas * (FOURPI * p->P / p->C) * dH;
      uc[k] = v[k] + d4 / (2.0 * rho);
    }
    const int it2 = or_absorption_cell(p, dt, sa, rho, uc, r4, Tn, I4, &T4);
    it = it2 > 0 ? (it2 > it ? it2 : it) : it2;
  }
  for (int m = 0; m < N; ++m) r5[m] = I4[m] + (to5 ? dFc[m] : 0.0);
  const int st = or_scattering_cell(p, dt, ss, vt, r5, Inew);
  double H4[3] = {0, 0, 0}, Hr4[3] = {0, 0, 0}, H5[3] = {0, 0, 0}, Hr5[3] = {0, 0, 0};
  for (int m = 0; m < N; ++m) {
    const double *n = p->mu + 3 * m;
    for (int k = 0; k < 3; ++k) {
      H4[k] += n[k] * p->w[m] * I4[m];
      Hr4[k] += n[k] * p->w[m] * r4[m];
      H5[k] += n[k] * p->w[m] * Inew[m];
      Hr5[k] += n[k] * p->w[m] * r5[m];
    }
  }
  const double cv = rho * p->R / (p->gamma - 1.0);
  const double dET = cv * (T4 - Tn);
  double m0sq = 0, m1sq = 0;
  for (int k = 0; k < 3; ++k) {
    const double d4 = -gas * (FOURPI * p->P / p->C) * (H4[k] - Hr4[k]);
    const double d5 = -gas * (FOURPI * p->P / p->C) * (H5[k] - Hr5[k]);
    dMom[k] = d4 + d5;
    const double m0 = rho * v[k];
    m0sq += m0 * m0;
    m1sq += (m0 + dMom[k]) * (m0 + dMom[k]);
  }
  *dEkin = (m1sq - m0sq) / (2.0 * rho);
  *dEgas = dET + *dEkin;
  *Tnew = T4;
  if (st != 0) return -1;
  return it;
}

/* Per-cell fields gathered from the field arrays. */
static void gather3(const double *a, long long nc, long long c, double *out) {
  out[0] = a[c];
  out[1] = a[nc + c];
  out[2] = a[2 * nc + c];
}

int or_step(const or_problem *p, double dt, const double *rho,
            const double *sa, const double *ss, const double *v,
            const double *I_in, double *I_out, double *T, double *dEgas,
            double *dEkin, double *dMom, double *E, double *F, double *Pr,
            int accumulate) {
  const long long nc = ncell_of(p);
  const int N = p->nang;
  /* Moments of I^n: J for the IV term, E, F, P_r for the velocity estimate. */
  double *En = (double *)malloc(sizeof(double) * nc);
  double *Fn = (double *)malloc(sizeof(double) * 3 * nc);
  double *Pn = (double *)malloc(sizeof(double) * 6 * nc);
  double *J = (double *)malloc(sizeof(double) * nc);
  double *dF = (double *)malloc(sizeof(double) * (size_t)N * nc);
  or_moments(p, I_in, En, Fn, Pn);
  for (long long c = 0; c < nc; ++c) J[c] = En[c] / FOURPI;
  /* Step 2: transport increments. */
  or_transport(p, dt, I_in, J, v, sa, ss, dF);
  int worst = 0, fail = 0;
#pragma omp parallel reduction(max : worst) reduction(| : fail)
  {
    double *buf = (double *)malloc(sizeof(double) * 6 * N);
    double *In = buf + 3 * N, *dFc = buf + 4 * N, *Inew = buf + 5 * N;
#pragma omp for schedule(static)
    for (long long c = 0; c < nc; ++c) {
      double vc[3], Fc[3], Pd[3], vt[3], dM[3], dEg, dEk, Tn1;
      gather3(v, nc, c, vc);
      gather3(Fn, nc, c, Fc);
      gather3(Pn, nc, c, Pd);
      /* Step 3: half-step velocity estimate from the moments of I^n. */
      vtilde_cell(p, dt, rho[c], sa[c] + ss[c], vc, Fc, En[c], Pd, vt);
      for (int m = 0; m < N; ++m) {
        In[m] = I_in[(long long)m * nc + c];
        dFc[m] = dF[(long long)m * nc + c];
      }
      const int it = source_cell(p, dt, rho[c], sa[c], ss[c], vc, vt, In, dFc, T[c], Inew,
                                 &Tn1, &dEg, &dEk, dM, buf);
      if (it < 0) fail = 1;
      if (it > worst) worst = it;
      T[c] = Tn1;
      for (int m = 0; m < N; ++m) I_out[(long long)m * nc + c] = Inew[m];
      if (dEkin) dEkin[c] = (accumulate ? dEkin[c] : 0.0) + dEk;
      if (accumulate) {
        dEgas[c] += dEg;
        for (int k = 0; k < 3; ++k) dMom[(long long)k * nc + c] += dM[k];
      } else {
        dEgas[c] = dEg;
        for (int k = 0; k < 3; ++k) dMom[(long long)k * nc + c] = dM[k];
      }
    }
    free(buf);
  }
  or_moments(p, I_out, E, F, Pr);
  free(En);
  free(Fn);
  free(Pn);
  free(J);
  free(dF);
  return fail ? -1 : worst;
}

int or_step_cells(const or_problem *p, double dt, const double *rho,
                  const double *sa, const double *ss, const double *v,
                  const double *I_in, const double *T_in, int ncsel,
                  const long long *cells, double *I_out, double *T_out,
                  double *dEgas, double *dEkin, double *dMom, double *E,
                  double *F, double *Pr) {
  const long long nc = ncell_of(p);
  const int N = p->nang;
  double *En = (double *)malloc(sizeof(double) * nc);
  double *Fn = (double *)malloc(sizeof(double) * 3 * nc);
  double *Pn = (double *)malloc(sizeof(double) * 6 * nc);
  double *J = (double *)malloc(sizeof(double) * nc);
  or_moments(p, I_in, En, Fn, Pn);
  for (long long c = 0; c < nc; ++c) J[c] = En[c] / FOURPI;
  int worst = 0, fail = 0;
#pragma omp parallel reduction(max : worst) reduction(| : fail)
  {
    double *buf = (double *)malloc(sizeof(double) * 6 * N);
    double *In = buf + 3 * N, *dFc = buf + 4 * N, *Inew = buf + 5 * N;
#pragma omp for schedule(dynamic, 4)
    for (int s = 0; s < ncsel; ++s) {
      const long long c = cells[s];
      const int x = (int)(c % p->n[0]);
      const int y = (int)((c / p->n[0]) % p->n[1]);
      const int z = (int)(c / ((long long)p->n[0] * p->n[1]));
      double vc[3], Fc[3], Pd[3], vt[3], dM[3], dEg, dEk, Tn1;
      gather3(v, nc, c, vc);
      gather3(Fn, nc, c, Fc);
      gather3(Pn, nc, c, Pd);
      vtilde_cell(p, dt, rho[c], sa[c] + ss[c], vc, Fc, En[c], Pd, vt);
      for (int m = 0; m < N; ++m) {
        In[m] = I_in[(long long)m * nc + c];
        dFc[m] = cell_dF(p, dt, I_in, J, v, sa, ss, m, x, y, z);
      }
      const int it = source_cell(p, dt, rho[c], sa[c], ss[c], vc, vt, In, dFc, T_in[c], Inew,
                                 &Tn1, &dEg, &dEk, dM, buf);
      if (it < 0) fail = 1;
      if (it > worst) worst = it;
      T_out[c] = Tn1;
      dEgas[c] = dEg;
      if (dEkin) dEkin[c] = dEk;
      double J1 = 0, H1[3] = {0, 0, 0}, K1[6] = {0, 0, 0, 0, 0, 0};
      for (int m = 0; m < N; ++m) {
        const double *n = p->mu + 3 * m;
        const double Iw = Inew[m] * p->w[m];
        I_out[(long long)m * nc + c] = Inew[m];
        J1 += Iw;
        for (int k = 0; k < 3; ++k) H1[k] += n[k] * Iw;
        K1[0] += n[0] * n[0] * Iw;
        K1[1] += n[1] * n[1] * Iw;
        K1[2] += n[2] * n[2] * Iw;
        K1[3] += n[0] * n[1] * Iw;
        K1[4] += n[0] * n[2] * Iw;
        K1[5] += n[1] * n[2] * Iw;
      }
      E[c] = FOURPI * J1;
      for (int k = 0; k < 3; ++k) {
        dMom[(long long)k * nc + c] = dM[k];
        F[(long long)k * nc + c] = FOURPI * H1[k];
      }
      for (int k = 0; k < 6; ++k) Pr[(long long)k * nc + c] = FOURPI * K1[k];
    }
    free(buf);
  }
  free(En);
  free(Fn);
  free(Pn);
  free(J);
  return fail ? -1 : worst;
}

/* ---------------------------------------------------------------- totals */
typedef struct {
  double s, c;
} ksum;

/* Neumaier compensated summation. */
static void kadd(ksum *k, double x) {
  const double t = k->s + x;
  if (fabs(k->s) >= fabs(x))
    k->c += (k->s - t) + x;
  else
    k->c += (x - t) + k->s;
  k->s = t;
}

void or_totals(const or_problem *p, const double *rho, const double *T,
               const double *E, const double *F, const double *dEgas,
               const double *dEkin, const double *dMom, const double *I,
               double *tot) {
  const long long nc = ncell_of(p);
  double vol = 1.0;
  for (int d = 0; d < p->ndim; ++d) vol *= p->dx[d];
  ksum k[10];
  memset(k, 0, sizeof(k));
  const double cvf = p->R / (p->gamma - 1.0);
  for (long long c = 0; c < nc; ++c) {
    kadd(&k[0], p->P * E[c] * vol);
    kadd(&k[1], cvf * rho[c] * T[c] * vol);
    kadd(&k[2], (dEgas ? dEgas[c] : 0.0) * vol);
    kadd(&k[3], (dEkin ? dEkin[c] : 0.0) * vol);
    for (int j = 0; j < 3; ++j) {
      kadd(&k[4 + j], (dMom ? dMom[(long long)j * nc + c] : 0.0) * vol);
      kadd(&k[7 + j], p->P / p->C * F[(long long)j * nc + c] * vol);
    }
  }
  for (int j = 0; j < 10; ++j) tot[j] = k[j].s + k[j].c;
  double mn = DBL_MAX;
  if (I)
    for (long long i = 0; i < (long long)p->nang * nc; ++i)
      if (I[i] < mn) mn = I[i];
  tot[10] = I ? mn : 0.0;
  tot[11] = 0.0;
}
