/*
 * rt.h -- C ABI of the MI355X (gfx950) radiative-transfer step library.
 *
 * The library advances the frequency-integrated specific intensity
 * I(x, n_m) on a Cartesian grid of discrete ordinates by the method of
 * Jiang, Stone & Davis (2014, ApJS 213, 7), one time step at a time:
 *   - explicit conservative upwind transport along every ray with
 *     monotonic piecewise-linear (van Leer) interface values, the
 *     optical-depth-reduced transport speed alpha*C for I - IV/C and the
 *     flow speed for IV = 3 n.v J (Section 4.2);
 *   - the half-step velocity estimate (Section 4.5);
 *   - the implicit absorption step in the mixed frame to O(v/c), coupled to
 *     the gas temperature (Section 4.3, Eq. absorptionmatrix);
 *   - the implicit scattering step (Section 4.4);
 *   - the angular quadrature (Section 3) giving E_r, F_r, P_r and the gas
 *     energy and momentum source terms (Sections 4.3-4.4, Step 7).
 * The gas (MHD) update is not part of the library: density, opacities and
 * velocity are inputs held fixed; the gas temperature is advanced.
 *
 * Units are the paper's dimensionless ones (Section 2): c is Crat, prat is
 * Prat, the equilibrium intensity is T^4/(4 pi).  Angle weights sum to 1,
 * so E_r = 4 pi sum W I, F_r = 4 pi sum W n I, P_r = 4 pi sum W n n I.
 *
 * Memory layout (all device arrays are caller-owned unless stated):
 *   - cell index c = x + nx*(y + ny*z);
 *   - per-cell scalars: [ncell] doubles;
 *   - vectors (v, F_r, dMom): [3][ncell] doubles (component-major);
 *   - pressure tensor P_r: [6][ncell] doubles, order xx, yy, zz, xy, xz, yz;
 *   - intensities I and transport increments dF: [nang][ncell] in the
 *     storage type of the context (double for RT_FP64, float for
 *     RT_FP32_MIXED): one contiguous plane of cells per angle.
 *
 * Calls are asynchronous on the given stream (a hipStream_t passed as a
 * void pointer; NULL is the default stream).  A context is not thread safe:
 * use one context per stream.  Every call returns an rt_status; device-side
 * failures (Newton non-convergence, non-finite or non-positive temperature)
 * set a flag that the next rt_sync_status() reports.  No exceptions cross
 * this interface.
 */
#ifndef RT_H
#define RT_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rt_status {
  RT_PENDING = 1,      /* (serving) the request has not completed yet        */
  RT_OK = 0,
  RT_EINVAL = -1,      /* invalid argument                                  */
  RT_ENOMEM = -2,      /* device or host allocation failed                  */
  RT_EDEVICE = -3,     /* HIP runtime error                                 */
  RT_ECFL = -4,        /* dt violates sum_d C |mu_d| dt / dx_d <= 1 (C the
                          reduced speed when the context has one)           */
  RT_ENOCONV = -5,     /* Newton iteration of the temperature did not
                          converge, or gave a non-positive/non-finite T     */
  RT_EBADQUAD = -6,    /* weights do not sum to 1 or |n| != 1               */
  RT_ESTATE = -7,      /* call order violated (e.g. no intensity bound)     */
  RT_EUNSUPPORTED = -8, /* valid request the library does not support       */
  RT_ETOOBIG = -9      /* (rt_step_static) the problem's scratch exceeds
                          RT_STATIC_SCRATCH_BYTES                           */
} rt_status;

enum { RT_BC_PERIODIC = 0, RT_BC_FIXED = 1, RT_BC_COPY = 2, RT_BC_VACUUM = 3 };
enum { RT_FP64 = 0, RT_FP32_MIXED = 1 };
enum { RT_QUAD_GAUSS_LEGENDRE = 0, RT_QUAD_LEVEL_SYMMETRIC = 1 };
/* Flag: use the half-step velocity estimate of Section 4.5 (default on). */
#define RT_ESTIMATE_V 1u
/* Flag: gas feedback (Section 4.1 Step 7 with the density held fixed):
 * after every step the gas momentum change of the step moves the flow,
 * v <- v + d(rho v)/rho, in rt_fields.v, and the next step's interface flow
 * speeds and IV follow (Section 5.2, equilibrium in a moving medium).  Angle
 * sets of at most 320 directions; not for served requests. */
#define RT_GAS_FEEDBACK 2u
/* Flag: the original transport that Section 4.2 starts from (Stone &
 * Mihalas 1992): every interface at speed C (alpha = 1) and I itself
 * upwinded, with no IV split.  Section 5.5 shows its numerical diffusion
 * swamping the physical diffusion in optically thick media; kept for that
 * comparison. */
#define RT_ORIGINAL_TRANSPORT 4u
/* Flag: second order in time for the absorption step.  Section 4.3 traces the
 * O(dt^2) gap between the gas energy change (Delta E_T + Delta E_K) and the
 * radiation energy change to the single solve of the absorption system and
 * names solving it twice as the remedy.  Reading: the system is solved at
 * the step's velocity u (the Step 3 estimate, or v), the Step 4 momentum
 * change d4 of that solution gives the time-centred velocity
 * v + d4/(2 rho), and the system is solved again at that velocity from the
 * same right-hand side and T^n; the second solution is the step's.  The
 * scattering step keeps u.  rt_step runs both solves in its fused kernel
 * (about 1.2 times the single-solve step), also with RT_GAS_FEEDBACK;
 * rt_source_implicit runs the step per cell, and returns RT_EUNSUPPORTED
 * when RT_GAS_FEEDBACK is set too. */
#define RT_SECOND_ORDER 8u
/* Number of entries of the totals vector. */
#define RT_NTOT 12

typedef struct rt_ctx rt_ctx;

typedef struct rt_grid {
  int ndim;      /* 1, 2 or 3; transport along the first ndim axes        */
  int n[3];      /* cells per axis, >= 1; unused axes must be 1           */
  double dx[3];  /* cell sizes (> 0 on active axes)                        */
  int bc[3][2];  /* RT_BC_* per axis and side (0 = low face); periodic on
                    one side requires periodic on the other               */
} rt_grid;

typedef struct rt_angles { /* host arrays, copied by rt_create */
  int n;                   /* number of directions, 1..RT_MAX_ANGLES       */
  const double *mu;        /* [n][3] direction cosines, |n| = 1            */
  const double *w;         /* [n] weights > 0 with sum 1                   */
} rt_angles;

#define RT_MAX_ANGLES 1024

typedef struct rt_params {
  double c;            /* Crat > 0                                          */
  double prat;         /* Prat >= 0                                         */
  double gamma;        /* adiabatic index > 1                               */
  double r_ideal;      /* ideal gas constant > 0; c_v = rho r/(gamma - 1)   */
  int precision;       /* RT_FP64 or RT_FP32_MIXED                          */
  unsigned flags;      /* RT_ESTIMATE_V | RT_GAS_FEEDBACK |
                          RT_ORIGINAL_TRANSPORT | RT_SECOND_ORDER           */
  double newton_rtol;  /* relative tolerance of the temperature Newton
                          iteration (e.g. 1e-14); <= 0 selects 1e-14        */
  int newton_maxit;    /* iteration limit (e.g. 64); <= 0 selects 64        */
  double c_reduced;    /* reduced speed of light 0 < c_reduced <= c, or 0 for
                          c itself (Section 6 combines the method with the
                          reduced-speed-of-light approximation): the
                          radiation advances at c_reduced (transport and
                          both implicit source steps take the time step
                          dt c_reduced/c, the CFL limit likewise) while the
                          gas exchanges energy and momentum at the true
                          rate (its changes are c/c_reduced times those of
                          the radiation), so steady states are those of c
                          and (c/c_reduced) Prat E_r + e_gas is conserved.
                          The O(v/c) factors keep c.  RT_EUNSUPPORTED with
                          RT_ESTIMATE_V (the velocity estimate is derived
                          for one speed).                                    */
} rt_params;

typedef struct rt_fields { /* device arrays, [ncell] doubles unless noted */
  const double *sigma_a;   /* absorption coefficient >= 0                  */
  const double *sigma_s;   /* scattering coefficient >= 0                  */
  const double *rho;       /* density > 0                                  */
  double *T;               /* gas temperature, read at time n and
                              overwritten with T^{n+1}                     */
  double *v;               /* [3][ncell] flow velocity: held fixed, or
                              updated in place with RT_GAS_FEEDBACK        */
} rt_fields;

typedef struct rt_out { /* device arrays; any pointer may be NULL */
  double *Er;           /* [ncell]    E_r of the new intensities           */
  double *Fr;           /* [3][ncell] F_r                                  */
  double *Pr;           /* [6][ncell] P_r                                  */
  double *dEgas;        /* [ncell] gas energy change (internal + kinetic)
                           summed over the steps of the call               */
  double *dMom;         /* [3][ncell] gas momentum change, summed likewise */
  double *totals;       /* [RT_NTOT] domain totals times the cell volume:
                           [0] Prat sum E_r, [1] sum c_v T, [2] sum dEgas,
                           [3] sum of the kinetic part of dEgas,
                           [4..6] sum dMom, [7..9] (Prat/c) sum F_r,
                           [10] min over cells and angles of I,
                           [11] largest Newton iteration count            */
} rt_out;

/* Angle sets (host only, Section 3).  kind RT_QUAD_GAUSS_LEGENDRE: order =
 * number of nodes (even, >= 2), directions (mu, 0, 0) for 1D slabs, weights
 * halved to sum 1.  kind RT_QUAD_LEVEL_SYMMETRIC: order N even in [2, 16],
 * N(N+2) directions with levels mu_i^2 = (6i - 5)/(3(N - 1)) (N = 4 gives
 * the cosines 1/3 and 0.882 printed in Section 5.2) and permutation-class
 * weights from the sphere averages of the symmetric even monomials.
 * Directions are written to mu[3*i + k], weights to w[i], for at most cap
 * directions.  Returns the number of directions, or a negative rt_status. */
int rt_quadrature(int kind, int order, double *mu, double *w, int cap);

/* Creates a context on the current HIP device for the problem Section 2 states
 * (the transfer equation on a Cartesian grid of discrete ordinates, with the
 * gas given by density, temperature, velocity and the two opacities) and
 * Section 3 discretises (directions n_m with weights W_m): validates the
 * grid, the angle
 * set (sum w = 1 within 1e-12; |n| = 1 within 1e-12 on 2D/3D grids, |n| <= 1
 * on 1D slabs, whose directions may be azimuthal averages (mu, 0, 0)) and the
 * parameters, copies the angle table to the device and allocates the
 * library-owned scratch: double-buffered per-cell moment fields (E, F, P and
 * 3 v J), the per-call interface table (alpha, flow speed), per-block partial
 * totals and a status word.  *out receives the context, or NULL on failure. */
int rt_create(const rt_grid *g, const rt_angles *a, const rt_params *p, rt_ctx **out);

/* Frees the context and its scratch (synchronises the device first). */
int rt_destroy(rt_ctx *ctx);

/* Binds two caller-owned device buffers of nang*ncell elements of the
 * storage type (layout [nang][ncell]); I_a holds the current state.  The library ping-pongs
 * between them; rt_current_intensity tells which one is current. */
int rt_bind_intensity(rt_ctx *ctx, void *I_a, void *I_b);
int rt_current_intensity(rt_ctx *ctx, void **I_cur);

/* Ghost intensities for an RT_BC_FIXED face: host array [nang] (beams,
 * inflow).  Section 4.1 Step 2 transports I through ghost zones; the
 * paper's tests fix them to injected beams and background inflow (Sections
 * 5.4 and 5.8).  Ghost zones are two cells deep and both layers take the
 * table; the ghost values of J, v and the opacities copy the edge cell.
 * Synchronises the device before the upload, so steps already queued on any
 * stream read the previous table and later steps the new one.  RT_EINVAL
 * for a bad axis or side or a face that is not RT_BC_FIXED; RT_EDEVICE
 * when the copy fails. */
int rt_set_fixed_bc(rt_ctx *ctx, int axis, int side, const double *I_ghost);

/* Position-dependent ghost intensities for an RT_BC_FIXED face, for beams
 * that enter through part of a face (the crossing beams of Section 5.4):
 * host array [nang][nface], nface = ncell / n[axis], the face cells ordered
 * by the two other axes with the lower one fastest (axis 0: y + n[1] z;
 * axis 1: x + n[0] z; axis 2: x + n[0] y).  Both ghost layers take the
 * value of their face cell; the ghost values of J, v and the opacities copy
 * the edge cell, as with rt_set_fixed_bc.  The library copies the array
 * into device memory that it owns until rt_destroy; a later rt_set_fixed_bc
 * on the face replaces it by an angle table again.  Synchronises the device
 * when it replaces a table.  RT_EINVAL for a bad axis or side or a face that
 * is not RT_BC_FIXED; RT_ENOMEM when the table cannot be allocated;
 * RT_EDEVICE when the copy fails. */
int rt_set_fixed_bc_face(rt_ctx *ctx, int axis, int side, const double *I_ghost);

/* Angular moments of the current intensities (Section 3) into out->Er, Fr,
 * Pr, and into the context's moment fields used by the next step. */
int rt_moments(rt_ctx *ctx, rt_out *out, void *stream);

/* Step 2 alone: writes the transport increment dF [nang][ncell] (storage
 * type) of the current intensities for time step dt (Section 4.2). */
int rt_transport(rt_ctx *ctx, double dt, const rt_fields *f, void *dF, void *stream);

/* Steps 3-5 and 7 alone: from the current intensities and dF (NULL = no
 * transport), computes the new intensities into the other bound buffer
 * (which becomes current), T^{n+1}, the moments and the gas source terms of
 * one step.  rt_transport followed by rt_source_implicit equals rt_step
 * with nsteps = 1. */
int rt_source_implicit(rt_ctx *ctx, double dt, const rt_fields *f, const void *dF,
                       rt_out *out, void *stream);

/* nsteps fused steps of the operator-split update of Section 4.1 (Steps 2-5
 * and the gas source terms of Step 7): transport (Section 4.2), velocity
 * estimate (Section 4.5), absorption (Section 4.3), scattering (Section 4.4)
 * and quadrature (Section 3); I read and written once per step.  RT_ECFL
 * when dt breaks the transport limit; RT_ESTATE without bound
 * intensities.  out->dEgas and
 * out->dMom receive the sums over the nsteps steps; the moments and totals
 * are those after the last step. */
int rt_step(rt_ctx *ctx, double dt, int nsteps, const rt_fields *f, rt_out *out,
            void *stream);

/* Library scratch per GPU of rt_step_static, in bytes (64 MiB): a device
 * array that each GPU the library runs on holds until the process ends. */
#define RT_STATIC_SCRATCH_BYTES (64ull << 20)

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the
 * sequence rt_create, rt_bind_intensity(I_a, I_b), rt_step(nsteps),
 * rt_destroy as one call that allocates nothing.  The library scratch the
 * context would allocate (angle tables, two moment fields, the interface
 * table, partial totals) is carved from a file-scope device array of
 * RT_STATIC_SCRATCH_BYTES per GPU instead, so a problem fits when it needs
 * about 282 bytes per cell plus 300 per direction (64^3 cells does not; 60^3
 * does); larger ones return RT_ETOOBIG before any device work.  Arguments,
 * layouts and results are those of the calls it stands for: I_a holds the
 * current intensities on entry; after the call the newest are in I_a when
 * nsteps is even and in I_b when it is odd.  Fixed faces take zero inflow
 * (the call has no ghost tables).  status is a caller-owned device int that
 * a step ORs with 1 when the temperature iteration fails (what rt_sync_status
 * reports for a context); the caller clears it.  Every call on a GPU shares
 * that GPU's array, whose contents the last call leaves behind: calls that
 * overlap on one GPU (other threads, or streams that run concurrently) race,
 * and are the caller's to order.  Errors as rt_create and rt_step, plus
 * RT_ETOOBIG. */
int rt_step_static(const rt_grid *g, const rt_angles *a, const rt_params *p, void *I_a,
                   void *I_b, double dt, int nsteps, const rt_fields *f, rt_out *out,
                   int *status, void *stream);

/* Fills the intensity buffer I ([nang][ncell], storage type) with the
 * equilibrium intensity T^4/(4 pi) of the device temperatures T ([ncell]
 * doubles) in every direction (Section 2, code units), on the stream. */
int rt_equilibrium_intensity(rt_ctx *ctx, const double *T, void *I, void *stream);

/* Waits for the context's work and reports (then clears) the device status:
 * RT_OK or RT_ENOCONV. */
int rt_sync_status(rt_ctx *ctx);

/* Kernel timing: when enabled, every fused-step launch is bracketed by HIP
 * events on its stream; rt_profile_read (which synchronises) returns the
 * summed duration in milliseconds and the launch count since the last
 * read, then resets them. */
int rt_profile_enable(rt_ctx *ctx, int enable);
int rt_profile_read(rt_ctx *ctx, double *total_ms, int *launches);

/* Static description of the context: number of angles, cells, bytes per
 * stored intensity, and the launch shape of the fused kernel. */
typedef struct rt_info {
  int nang;
  long long ncell;
  int storage_bytes;
  int block_threads;
  long long grid_blocks;
} rt_info;
int rt_get_info(rt_ctx *ctx, rt_info *info);

/* Human-readable text of an rt_status. */
const char *rt_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif
