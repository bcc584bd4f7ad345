/*
 * Plain FP64 CPU oracle of one time step of the time-dependent,
 * frequency-integrated radiative transfer method of Jiang, Stone & Davis
 * (2014), "An Algorithm for Radiation Magnetohydrodynamics Based on Solving
 * the Time-dependent Transfer Equation" (ApJS 213, 7; arXiv:1403.6126).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the reference against which the
 * GPU library is checked; it shares no code, header, table or helper with
 * the GPU path.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It is written for clarity, not speed.
 *
 * Conventions: cell index x + nx*(y + ny*z); intensities I[m*ncell + c]
 * (angle-major); velocity v[k*ncell + c]; pressure tensor components in the
 * order xx, yy, zz, xy, xz, yz.  Angle weights sum to one, so J = sum W I is
 * the mean intensity (E_r = 4 pi J, F_r = 4 pi H, P_r = 4 pi K in the
 * paper's dimensionless units, Section 2).
 */
#ifndef RT_ORACLE_H
#define RT_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_BC_PERIODIC = 0, OR_BC_FIXED = 1, OR_BC_COPY = 2, OR_BC_VACUUM = 3 };
enum { OR_NTOT = 12 };

typedef struct or_problem {
  int ndim;              /* 1, 2 or 3 active axes (transport only along them) */
  int n[3];              /* cells per axis; unused axes have n = 1            */
  double dx[3];          /* cell sizes                                        */
  int bc[3][2];          /* boundary code per axis and side (0 = low face)    */
  int nang;
  const double *mu;      /* [nang][3] direction cosines                       */
  const double *w;       /* [nang] weights, sum 1                             */
  const double *ghost[3][2]; /* [nang] ghost intensities for OR_BC_FIXED      */
  double C;              /* Crat: dimensionless speed of light                */
  double P;              /* Prat                                              */
  double gamma;          /* adiabatic index                                   */
  double R;              /* R_ideal                                           */
  int estimate_v;        /* 1: half-step velocity estimate (Section 4.5)      */
  double rtol;           /* Newton relative tolerance                         */
  int maxit;             /* Newton iteration limit                            */
  int original;          /* 1: the original transport of Stone & Mihalas 1992
                            that Section 4.2 starts from (speed C, I itself
                            upwinded, no IV split), as in the Section 5.5
                            comparison                                       */
  const double *ghost_face[3][2]; /* [nang][nface] position-dependent ghost
                            intensities of an OR_BC_FIXED face, or NULL for
                            its angle table; nface = cells of the face, in
                            order of the two other axes, lower one fastest
                            (beams through part of a face, Section 5.4)    */
  double chat;           /* reduced speed of light (0: C itself): the
                            radiation advances at chat, the gas exchanges
                            energy and momentum at the true rate (the
                            reduced-speed-of-light approximation that
                            Section 6 combines with the method)             */
  int second_order;      /* 1: the absorption system of Section 4.3 solved
                            twice per step, the second time with the
                            time-centred velocity of the first solution
                            (the second-order-in-time variant that section
                            names; see source_cell)                         */
} or_problem;

/* Angular quadrature of I (Section 3): E = 4pi sum W I, F_k = 4pi sum W mu_k I,
 * P_ij = 4pi sum W mu_i mu_j I.  Any output pointer may be NULL. */
void or_moments(const or_problem *p, const double *I, double *E, double *F,
                double *Pr);

/* Time step of the radiation for a step dt of the gas: dt chat/C with a
 * reduced speed of light chat, else dt. */
double or_radiation_dt(const or_problem *p, double dt);

/* Transport increment Delta F (Section 4.2) for every angle and cell, from
 * the intensities I and the mean intensity J (both at time n). */
void or_transport(const or_problem *p, double dt, const double *I,
                  const double *J, const double *v, const double *sa,
                  const double *ss, double *dF);

/* Half-step velocity estimate (Section 4.5), per cell. */
void or_vtilde(const or_problem *p, double dt, const double *rho,
               const double *sa, const double *ss, const double *v,
               const double *E, const double *F, const double *Pr,
               double *vt);

/* Implicit absorption sub-step (Section 4.3) of one cell: given the right-hand
 * side r[nang], the temperature Tn, the fixed velocity u[3] and the cell's
 * data, returns I'[nang] and T'.  Returns the Newton iteration count, or -1
 * when the iteration did not converge within maxit. */
int or_absorption_cell(const or_problem *p, double dt, double sa, double rho,
                       const double *u, const double *r, double Tn,
                       double *Iout, double *Tout);

/* Implicit scattering sub-step (Section 4.4) of one cell: dense solve of the
 * N x N system for the unknowns I_m W_m.  Returns 0, or -1 if singular. */
int or_scattering_cell(const or_problem *p, double dt, double ss,
                       const double *u, const double *r, double *Iout);

/* One full step (Steps 2-5 and the source terms of Step 7) for all cells.
 * I_in is I^n, I_out receives I^{n+1}; T is updated in place.  dEgas[c] and
 * dMom[3][c] receive the gas energy and momentum changes of this step
 * (added to the existing values when accumulate != 0).  E, F, Pr receive the
 * moments of I^{n+1} (may be NULL); dEkin (may be NULL) the kinetic part of
 * dEgas.  Returns the largest Newton iteration
 * count, or -1 if any cell failed to converge. */
int or_step(const or_problem *p, double dt, const double *rho,
            const double *sa, const double *ss, const double *v,
            const double *I_in, double *I_out, double *T, double *dEgas,
            double *dEkin, double *dMom, double *E, double *F, double *Pr,
            int accumulate);

/* The same step restricted to the listed cells (every other output entry is
 * left untouched); I_out, T, dEgas, dMom, E, F, Pr are indexed by cell as
 * in or_step.  T is read from T_in and written to T_out. */
int or_step_cells(const or_problem *p, double dt, const double *rho,
                  const double *sa, const double *ss, const double *v,
                  const double *I_in, const double *T_in, int ncsel,
                  const long long *cells, double *I_out, double *T_out,
                  double *dEgas, double *dEkin, double *dMom, double *E,
                  double *F, double *Pr);

/* Whole-domain totals (compensated sums, times the cell volume):
 * [0] P sum E, [1] sum c_v T, [2] sum dEgas, [3] sum dE_kin, [4..6] sum dMom,
 * [7..9] (P/C) sum F, [10] min I, [11] 0. */
void or_totals(const or_problem *p, const double *rho, const double *T,
               const double *E, const double *F, const double *dEgas,
               const double *dEkin, const double *dMom, const double *I,
               double *tot);

/* Number of OpenMP threads the oracle uses (1 when built without OpenMP). */
int or_threads(void);

/* Sets the number of OpenMP threads of the later calls (n >= 1). */
void or_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
