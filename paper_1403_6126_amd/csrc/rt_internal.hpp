// Host-side internals shared by the context API, the kernel launchers and
// the serving runtime: the context object, its device-memory plan, and the
// launch entry points of the step kernels (defined per storage precision in
// their own translation units).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <utility>
#include <vector>

#include "rt.h"
#include "rt_common.hpp"

namespace rtk {

// Launch shape of the step kernel of a context: waves > 0 selects the
// wave-group kernel (64 cells per block, `waves` waves, `groups` angle
// groups of kAnglesPerWave per wave); waves == 0 the thread-per-cell kernel.
constexpr int kAnglesPerWave = 10;
constexpr int kMaxGroupsPerWave = 4;
struct KShape {
  int waves = 0, groups = 0;
  bool periodic = true;
  bool second = false;  // second-order absorption (both solves in the step)
};

// One request of a packed persistent launch: a whole solve of nsteps steps
// for one grid that a single workgroup advances tile by tile.  a.I_in /
// a.mom_in hold the current state, a.I_out / a.mom_out the other buffers of
// the ping-pong; a.partials has kNtot rows of a.nparts = ceil(ncell/64).
struct PackedJob {
  StepArgs a;
  int nsteps;
  int pad_;
  double *totals;  // [kNtot] totals of the solve (nullable)
};

// Step launchers (defined in rt_kernels_f64.hip / rt_kernels_f32.hip).
hipError_t launch_step_f64(const StepArgs &a, const KShape &k, bool fused, long long blocks,
                           hipStream_t s);
hipError_t launch_step_f32(const StepArgs &a, const KShape &k, bool fused, long long blocks,
                           hipStream_t s);
// The wave-group kernels of one precision and number of groups per wave
// (rt_step3_<f64|f32>_g<1..4>.hip): fused, second-order fused (k.second) or
// source-only steps, and (FP32) the packed persistent launches.
#define RT_DECLARE_STEP3(suf, ng)                                                           \
  void launch_step3_##suf##_##ng(const StepArgs &a, const KShape &k, bool fused,            \
                                 long long blocks, hipStream_t s);                          \
  void launch_packed_##suf##_##ng(const PackedJob *jobs, int njobs, int waves, bool periodic, \
                                  hipStream_t s);
RT_DECLARE_STEP3(f64, 1)
RT_DECLARE_STEP3(f64, 2)
RT_DECLARE_STEP3(f64, 3)
RT_DECLARE_STEP3(f64, 4)
RT_DECLARE_STEP3(f32, 1)
RT_DECLARE_STEP3(f32, 2)
RT_DECLARE_STEP3(f32, 3)
RT_DECLARE_STEP3(f32, 4)
#undef RT_DECLARE_STEP3

// Packed persistent launches: one workgroup of 64*waves threads per job;
// every job of a launch has the launch shape (waves, groups) of its own
// context, so that it sums its angles in the order rt_step does, and the
// given boundary class.
hipError_t launch_packed_f64(const PackedJob *jobs, int njobs, int waves, int groups,
                             bool periodic, hipStream_t s);
hipError_t launch_packed_f32(const PackedJob *jobs, int njobs, int waves, int groups,
                             bool periodic, hipStream_t s);

}  // namespace rtk

// Context of one grid and angle set.
struct rt_ctx {
  rt_grid g;
  rt_params p;
  int nang = 0;
  long long ncell = 0;
  int device = 0;
  bool all_periodic = true;
  double cfl_sum = 0.0;  // max over angles of sum_d |mu_d| / dx_d
  std::vector<double> h_mu, h_w, h_ghost;
  std::vector<float> h_muf, h_wf;       // FP32 copies of the angle table
  // device memory: one block when carved from a caller's arena, else
  // separate hipMalloc allocations owned by the context
  bool owns_device = true;
  double *d_mu = nullptr, *d_w = nullptr, *d_ghost = nullptr;
  // position-dependent ghost tables of fixed faces (axis*2 + side), each its
  // own allocation owned by the context
  double *d_gface[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  float *d_muf = nullptr, *d_wf = nullptr;
  int nrec = 0;                         // angle records (nang, padded to the kernel's slots)
  double *d_arec = nullptr;             // [nrec][kRec] per-call angle records
  float *d_arecf = nullptr;
  void *I[2] = {nullptr, nullptr};
  int cur = 0;
  double *mom[2] = {nullptr, nullptr};  // [13][ncell]: E, F, P, 3vJ
  int mom_cur = 0;
  double *faces = nullptr;              // [3][3][ncell] interface table of the call
  rtk::KShape shape;
  bool mom_valid = false;
  double *partials = nullptr;           // [kNtot][nblocks], kept over the steps of a call
  int *status = nullptr;
  long long nblocks = 0;
  bool profile = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
  double prof_ms = 0.0;
  int prof_n = 0;
};

namespace rtk {

// Validates the arguments and fills the host part of a new context (no
// device calls).  Returns an rt_status.
int ctx_init_host(const rt_grid *g, const rt_angles *a, const rt_params *p, rt_ctx *c);
// Bytes of device scratch the context needs (tables, moments, interface
// table, partial totals, status word), 256-byte aligned.
size_t ctx_scratch_bytes(const rt_ctx *c);
// Points the context's scratch into base (ctx_scratch_bytes long) and
// uploads the tables / clears the counters on stream s.
int ctx_attach_scratch(rt_ctx *c, char *base, hipStream_t s);
// Steps k0 .. k1-1 of a call of ntotal steps whose interface table is
// already prepared: the accumulations restart at step 0 and the outputs are
// written at step ntotal-1, so consecutive ranges give the results of one
// rt_step call bit for bit.
int ctx_step_range(rt_ctx *c, double dt, const rt_fields *f, rt_out *o, int k0, int k1,
                   int ntotal, hipStream_t s);
// The body of rt_step for a bound context.
int ctx_step(rt_ctx *c, double dt, int nsteps, const rt_fields *f, rt_out *o, hipStream_t s);
// Moments of the current intensities into the context's moment fields.
int ctx_moments(rt_ctx *c, hipStream_t s);
// Interface table of a call (dt, fields) and 3 v J of the current moments.
int ctx_prepare_call(rt_ctx *c, double dt, const rt_fields *f, hipStream_t s);
// Fills the step arguments common to every launch of the context.
void ctx_fill_args(const rt_ctx *c, double dt, const rt_fields *f, StepArgs &a);
// I[m][c] = T[c]^4 / (4 pi) for every angle (storage type of the context).
int ctx_init_equilibrium(rt_ctx *c, const double *T, void *I, hipStream_t s);
long long ctx_step_blocks(const rt_ctx *c, bool fused);
int ctx_storage_bytes(const rt_ctx *c);
int ctx_check_dt(const rt_ctx *c, double dt);

}  // namespace rtk
