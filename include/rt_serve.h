/*
 * rt_serve.h -- serving runtime of the radiative-transfer step library:
 * independent solves (a grid, an angle set, fields, a time step and a
 * number of steps each) submitted from the host and run with continuous
 * batching on one GPU.
 *
 * Each solve is the method of rt.h (Sections 3-4 of Jiang, Stone & Davis
 * 2014): nsteps fused steps from the given intensities (or from the
 * equilibrium intensity T^4/(4 pi) in every direction), with the density,
 * opacities and velocity held fixed and the gas temperature advanced.
 *
 * Life of a request:
 *   - rt_serve_submit validates it (the checks of rt_create, the CFL limit)
 *     and queues it; the call does not wait for the GPU;
 *   - an IO thread admits queued requests in submission order when the
 *     server's HBM arena can hold the request's footprint (two intensity
 *     buffers of nang*ncell elements, the fields, the outputs and the
 *     step scratch) and fewer than max_active requests are admitted, then
 *     uploads its inputs;
 *   - a scheduler thread runs admitted requests concurrently: FP32-mixed
 *     requests of at most packed_cells cells are packed into persistent
 *     launches in which one workgroup advances a whole solve; every other
 *     request advances by chunks of about chunk_work cell-angle updates,
 *     at most two chunks in flight per request, on one of two streams: the
 *     requests of at least large_work updates per step run one at a time in
 *     submission order on the first, the others round-robin on the second,
 *     so that requests arriving while others run start at once and their
 *     work overlaps the large request on the device;
 *   - on completion the IO thread copies the results to the caller's host
 *     buffers and releases the arena memory.
 * A request's results do not depend on the other requests in flight: each
 * request runs the same kernels, with the same partition of its cells into
 * blocks, whatever else is admitted (the packed and the per-step launches
 * also agree with each other and with rt_step bit for bit).
 *
 * Threading: the functions below may be called from any host thread.  Host
 * input arrays of a request must stay valid until it completes; its output
 * arrays are written by the IO thread just before completion.
 */
#ifndef RT_SERVE_H
#define RT_SERVE_H

#include "rt.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rt_server rt_server;

typedef struct rt_serve_config {
  unsigned long long pool_bytes; /* HBM arena for admitted requests, > 0     */
  int max_active;                /* requests admitted at once, >= 1         */
  long long packed_cells;        /* FP32-mixed requests with ncell <= this
                                    run in packed persistent launches (0:
                                    never)                                  */
  long long chunk_work;          /* cell-angle updates per chunk, >= 1      */
  long long large_work;          /* updates per step from which a request
                                    uses the large-request stream, >= 1     */
} rt_serve_config;

typedef struct rt_request {
  rt_grid grid;
  rt_angles angles;        /* host arrays, copied by rt_serve_submit        */
  rt_params params;
  double dt;               /* time step (CFL-checked like rt_step)          */
  int nsteps;              /* >= 1                                          */
  const double *ghost;     /* [3][2][nang] ghost intensities of the
                              RT_BC_FIXED faces (axis, side), or NULL for
                              zeros; host, copied by rt_serve_submit        */
  /* host inputs, [ncell] doubles (v: [3][ncell]), read at admission       */
  const double *sigma_a, *sigma_s, *rho, *T, *v;
  const void *I0;          /* [nang][ncell] initial intensities in the
                              storage type, or NULL for T^4/(4 pi)          */
  /* host outputs, written at completion; any may be NULL                  */
  double *T_out;           /* [ncell] T after the last step                 */
  double *Er;              /* [ncell] E_r after the last step               */
  double *Fr;              /* [3][ncell] F_r after the last step            */
  double *totals;          /* [RT_NTOT] as rt_out.totals of rt_step         */
  void *I_out;             /* [nang][ncell] final intensities (storage type) */
} rt_request;

typedef struct rt_serve_result {
  int status;      /* RT_OK, RT_ENOCONV (device status of the solve), or the
                      error that stopped it                                 */
  int packed;      /* 1 when it ran inside a packed persistent launch       */
  double t_submit; /* seconds on the server clock (steady, zero at create)  */
  double t_admit;
  double t_done;   /* results visible in the host output arrays             */
} rt_serve_result;

typedef struct rt_serve_counters {
  long long submitted, completed, active, peak_active;
  unsigned long long pool_bytes, pool_used, peak_pool_used;
  long long packed_launches, packed_requests, chunk_launches;
  double cell_angle_updates; /* sum of ncell*nang*nsteps of completed ones */
} rt_serve_counters;

/* Creates a server on the current HIP device: allocates the arena, the
 * streams and the staging of the packed launches, and starts the two host
 * threads.  Returns RT_EINVAL for a bad configuration (before any device
 * call), RT_ENOMEM when the arena cannot be allocated. */
int rt_serve_create(const rt_serve_config *cfg, rt_server **out);

/* Validates and queues a request; *id receives its handle.  RT_ENOMEM when
 * its footprint exceeds the whole arena. */
int rt_serve_submit(rt_server *s, const rt_request *r, long long *id);

/* RT_PENDING while the request is in flight; RT_OK once complete, with
 * *res filled (res may be NULL).  RT_EINVAL for an unknown id. */
int rt_serve_poll(rt_server *s, long long id, rt_serve_result *res);

/* Blocks until the request completes, then as rt_serve_poll. */
int rt_serve_wait(rt_server *s, long long id, rt_serve_result *res);

/* Seconds on the server clock. */
double rt_serve_now(rt_server *s);

int rt_serve_get_counters(rt_server *s, rt_serve_counters *c);

/* Waits for every submitted request, stops the threads and frees the
 * server's device and host memory. */
int rt_serve_destroy(rt_server *s);

#ifdef __cplusplus
}
#endif
#endif
