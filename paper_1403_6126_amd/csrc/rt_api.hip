// Host side of the context API declared in include/rt.h: validation,
// device-memory plan, and the launches of the per-call and per-step kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "rt.h"
#include "rt_cellwise.hpp"
#include "rt_internal.hpp"

namespace rtk {

// Interface table, per-call angle factors and IV basis (once per call).
// faces[(d*3 + j)*ncell + c] for the face between the cell below c along
// axis d (wrapped; the edge cell itself at a non-periodic low boundary,
// whose ghost copies it) and c, with the face opacity and flow speed u the
// means of the two cells (Section 4.2):
//   j = 0  C alpha, the transport speed factor times C;
//   j = 1  the lower cell's share of the centred IV value: 1 when the flow
//          goes up the axis (u > 0, upwind = lower cell), 0 when it goes
//          down, 1/2 at u = 0 (centred);
//   j = 2  the signed van Leer factor of the IV value, sign(u) (1 - nu_v),
//          nu_v = |u| dt/dx (0 at u = 0).
// arec[m*kRec + f] (FP64, and FP32 copies) are the per-angle records of the
// call: direction, 1 - C |mu_d| dt/dx_d, w, w n_d, w n_i n_j and the sign
// bits of the direction (as integers in the slot's low word); records
// nang .. nrec-1 (the padding slots of the wave-group kernel) are zero.
// wv = 3 v E/(4pi) of the current moments into mom[10..12].  One thread per
// cell and per record (max of the two).
__global__ __launch_bounds__(kBlock) void k_faces(StepArgs p, double *faces, double *mom,
                                                  double *arec, float *arecf, int nrec) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c < nrec) {
    double r[kRec];
    for (int f = 0; f < kRec; ++f) r[f] = 0.0;
    if (c < p.nang) {
      const double n[3] = {p.mu[c], p.mu[p.nang + c], p.mu[2 * p.nang + c]};
      const double w = p.w[c];
      for (int d = 0; d < 3; ++d) {
        r[rec_n0 + d] = n[d];
        r[rec_h0 + d] = 1.0 - p.C * fabs(n[d]) * p.dt_dx[d];
        r[rec_wn0 + d] = w * n[d];
      }
      r[rec_w] = w;
      r[rec_wnn + 0] = w * n[0] * n[0];
      r[rec_wnn + 1] = w * n[1] * n[1];
      r[rec_wnn + 2] = w * n[2] * n[2];
      r[rec_wnn + 3] = w * n[0] * n[1];
      r[rec_wnn + 4] = w * n[0] * n[2];
      r[rec_wnn + 5] = w * n[1] * n[2];
    }
    // the signs of the direction as integer bits (the step kernel tests
    // them on the scalar unit, which has no floating-point compare)
    unsigned flags = 0;
    for (int d = 0; d < 3; ++d) {
      if (r[rec_n0 + d] > 0.0) flags |= 1u << d;
      if (r[rec_n0 + d] != 0.0) flags |= 8u << d;
    }
    for (int f = 0; f < kRec; ++f) {
      if (f == rec_flags) {
        unsigned long long bits = flags;
        arec[(size_t)c * kRec + f] = __longlong_as_double((long long)bits);
        arecf[(size_t)c * kRec + f] = __uint_as_float(flags);
      } else {
        arec[(size_t)c * kRec + f] = r[f];
        arecf[(size_t)c * kRec + f] = float(r[f]);
      }
    }
  }
  if (c >= p.ncell) return;
  const size_t N = (size_t)p.ncell;
  const double sig_c = p.sa[c] + p.ss[c];
  const int q[3] = {c % p.n[0], (c / p.n[0]) % p.n[1], c / (p.n[0] * p.n[1])};
  for (int d = 0; d < p.ndim; ++d) {
    int cl;
    if (q[d] > 0)
      cl = c - p.stride[d];
    else if (p.bc[d][0] == kPeriodic)
      cl = c + (p.n[d] - 1) * p.stride[d];
    else
      cl = c;
    const double sig = 0.5 * ((p.sa[cl] + p.ss[cl]) + sig_c);
    const double u = 0.5 * (p.v[(size_t)d * N + cl] + p.v[(size_t)d * N + c]);
    faces[(size_t)(d * 3 + 0) * N + c] = p.C * alpha_of(sig, p.dl10[d]);
    faces[(size_t)(d * 3 + 1) * N + c] = iv_lower_share(u);
    faces[(size_t)(d * 3 + 2) * N + c] = iv_signed_factor(u, p.dt_dx[d]);
  }
  const double J = mom[c] * (1.0 / kFourPi);
  for (int k = 0; k < 3; ++k) mom[(size_t)(10 + k) * N + c] = p.ivfac * p.v[(size_t)k * N + c] * J;
}

// Sets one int in device memory (status words; a kernel, not a memset, so
// that a captured graph replays it correctly).
__global__ void k_set_int(int *p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

__global__ __launch_bounds__(kVLanes) void k_totals(const double *partials, int nblocks,
                                                    double *out) {
  __shared__ double red[kNtot * kVWaves];
  totals_reduce(partials, nblocks, out, red);
}


// I[m][c] = T[c]^4 / (4 pi), the equilibrium intensity in every direction.
template <typename S>
__global__ __launch_bounds__(kBlock) void k_equilibrium(const double *T, S *I, int ncell,
                                                        int nang) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= ncell) return;
  const double t = T[c];
  const S b = S((t * t) * (t * t) / kFourPi);
  for (int m = 0; m < nang; ++m) I[(size_t)m * ncell + c] = b;
}

namespace {

bool hip_ok(hipError_t e) { return e == hipSuccess; }

// Kernel launches report failure through hipGetLastError only; an error left
// by an earlier call of this thread (already returned by that call) is
// cleared first so that the check after a launch sees only the launch.
void clear_stale_error() { (void)hipGetLastError(); }

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Waves per block of the wave-group kernel by storage type: the angle
// groups are dealt to at most this many waves (more groups per wave amortise
// the per-cell work of a wave over more angles), and to up to kMaxWaves when
// the groups would not fit kMaxGroupsPerWave per wave.
#ifndef RT_GROUP_WAVES_F64
#define RT_GROUP_WAVES_F64 4
#endif
#ifndef RT_GROUP_WAVES_F32
#define RT_GROUP_WAVES_F32 4
#endif

KShape pick_shape(int nang, bool periodic, int precision) {
  KShape k;
  k.periodic = periodic;
  const int ng = (nang + kAnglesPerWave - 1) / kAnglesPerWave;
  const int pref = precision == RT_FP32_MIXED ? RT_GROUP_WAVES_F32 : RT_GROUP_WAVES_F64;
  int G = ng < pref ? ng : pref;
  int NG = (ng + G - 1) / G;
  if (NG > kMaxGroupsPerWave) {
    G = ng < kMaxWaves ? ng : kMaxWaves;
    NG = (ng + G - 1) / G;
  }
  if (NG <= kMaxGroupsPerWave) {
    k.waves = G;
    k.groups = NG;
  }
  return k;
}

long long cell_blocks(const rt_ctx *c) { return (c->ncell + kBlock - 1) / kBlock; }

bool fields_ok(const rt_fields *f) {
  return f && f->sigma_a && f->sigma_s && f->rho && f->T && f->v;
}

void launch_step(const rt_ctx *c, const StepArgs &a, bool fused, hipStream_t s) {
  clear_stale_error();
  if (c->p.precision == RT_FP32_MIXED)
    launch_step_f32(a, c->shape, fused, ctx_step_blocks(c, fused), s);
  else
    launch_step_f64(a, c->shape, fused, ctx_step_blocks(c, fused), s);
}

void launch_transport(const rt_ctx *c, const StepArgs &a, hipStream_t s) {
  clear_stale_error();
  dim3 g((unsigned)cell_blocks(c)), b(kBlock);
  if (c->p.precision == RT_FP32_MIXED) {
    if (c->all_periodic)
      hipLaunchKernelGGL((k_transport<float, float, true>), g, b, 0, s, a);
    else
      hipLaunchKernelGGL((k_transport<float, float, false>), g, b, 0, s, a);
  } else {
    if (c->all_periodic)
      hipLaunchKernelGGL((k_transport<double, double, true>), g, b, 0, s, a);
    else
      hipLaunchKernelGGL((k_transport<double, double, false>), g, b, 0, s, a);
  }
}

void launch_moments(const rt_ctx *c, const StepArgs &a, hipStream_t s) {
  clear_stale_error();
  dim3 g((unsigned)cell_blocks(c)), b(kBlock);
  if (c->p.precision == RT_FP32_MIXED)
    hipLaunchKernelGGL(k_moments<float>, g, b, 0, s, a);
  else
    hipLaunchKernelGGL(k_moments<double>, g, b, 0, s, a);
}

int ensure_moments(rt_ctx *c, hipStream_t s) {
  if (c->mom_valid) return RT_OK;
  return ctx_moments(c, s);
}

hipEvent_t take_event(rt_ctx *c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// One step (fused or from a given dF); swaps the current buffers.
int one_step(rt_ctx *c, double dt, const rt_fields *f, const void *dF, bool fused, rt_out *o,
             bool first, bool last, hipStream_t s) {
  StepArgs a;
  ctx_fill_args(c, dt, f, a);
  a.I_in = c->I[c->cur];
  a.I_out = c->I[1 - c->cur];
  a.mom_in = c->mom[c->mom_cur];
  a.mom_out = c->mom[1 - c->mom_cur];
  a.dF_in = dF;
  a.nparts = (int)ctx_step_blocks(c, fused);
  a.accumulate = first ? 0 : 1;
  if (o) {
    a.dEgas = o->dEgas;
    a.dMom = o->dMom;
    if (last) {
      a.oE = o->Er;
      a.oF = o->Fr;
      a.oP = o->Pr;
    }
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c->profile && fused) {
    e0 = take_event(c);
    e1 = take_event(c);
    if (e0 && e1) hipEventRecord(e0, s);
  }
  launch_step(c, a, fused, s);
  if (!hip_ok(hipGetLastError())) return RT_EDEVICE;
  if (e0 && e1) {
    hipEventRecord(e1, s);
    c->pending.emplace_back(e0, e1);
  }
  if (last && o && o->totals) {
    hipLaunchKernelGGL(k_totals, dim3(1), dim3(kVLanes), 0, s, c->partials,
                       a.nparts, o->totals);
    if (!hip_ok(hipGetLastError())) return RT_EDEVICE;
  }
  c->cur = 1 - c->cur;
  c->mom_cur = 1 - c->mom_cur;
  c->mom_valid = true;
  return RT_OK;
}

}  // namespace

long long ctx_step_blocks(const rt_ctx *c, bool fused) {
  // the wave-group kernel works in tiles of 64 cells; a second-order step
  // from a given dF runs on the thread-per-cell kernel
  const bool tiles = c->shape.waves && (fused || !c->shape.second);
  return tiles ? (c->ncell + 63) / 64 : (c->ncell + kBlock - 1) / kBlock;
}

int ctx_storage_bytes(const rt_ctx *c) { return c->p.precision == RT_FP32_MIXED ? 4 : 8; }

// The speed at which the radiation advances: c, or the reduced speed.
double radiation_speed(const rt_ctx *c) {
  return c->p.c_reduced > 0.0 ? c->p.c_reduced : c->p.c;
}

int ctx_check_dt(const rt_ctx *c, double dt) {
  if (!(dt > 0.0) || !std::isfinite(dt)) return RT_EINVAL;
  if (radiation_speed(c) * dt * c->cfl_sum > 1.0 + 1e-12) return RT_ECFL;
  return RT_OK;
}

void ctx_fill_args(const rt_ctx *c, double dt_call, const rt_fields *f, StepArgs &a) {
  std::memset(&a, 0, sizeof(a));
  // with the reduced speed of light the radiation takes the step dt c_r/C in
  // every one of its terms (transport and sources); the gas keeps the true
  // coupling through a heat capacity (and, in the outputs, momentum) scaled
  // by c_r/C, which gives the temperature of the true-rate gas equation
  const double sc = radiation_speed(c) / c->p.c;
  const double dt = dt_call * sc;
  a.gasfac = 1.0 / sc;
  a.ndim = c->g.ndim;
  a.ivfac = (c->p.flags & RT_ORIGINAL_TRANSPORT) ? 0.0 : 3.0;
  for (int d = 0; d < 3; ++d) {
    a.n[d] = c->g.n[d];
    for (int s = 0; s < 2; ++s) a.bc[d][s] = c->g.bc[d][s];
    a.dt_dx[d] = dt / c->g.dx[d];
    // the original transport has alpha = 1 at every interface (zero length
    // scale in its optical depth) and no IV split (IV = 0, I~ = I)
    a.dl10[d] = (c->p.flags & RT_ORIGINAL_TRANSPORT) ? 0.0 : 10.0 * c->g.dx[d];
  }
  a.stride[0] = 1;
  a.stride[1] = c->g.n[0];
  a.stride[2] = c->g.n[0] * c->g.n[1];
  a.ncell = (int)c->ncell;
  a.nang = c->nang;
  a.dt = dt;
  a.C = c->p.c;
  a.invC = 1.0 / c->p.c;
  a.P = c->p.prat;
  a.cvfac = c->p.r_ideal / (c->p.gamma - 1.0) * sc;
  double vol = 1.0;
  for (int d = 0; d < c->g.ndim; ++d) vol *= c->g.dx[d];
  a.vol = vol;
  a.rtol = c->p.newton_rtol;
  a.maxit = c->p.newton_maxit;
  a.estimate_v = (c->p.flags & RT_ESTIMATE_V) ? 1 : 0;
  a.mu = c->d_mu;
  a.w = c->d_w;
  a.muf = c->d_muf;
  a.wf = c->d_wf;
  a.ghost = c->d_ghost;
  a.arec = c->d_arec;
  a.arecf = c->d_arecf;
  for (int f = 0; f < 6; ++f) a.gface[f] = c->d_gface[f];
  a.faces = c->faces;
  if (f) {
    a.sa = f->sigma_a;
    a.ss = f->sigma_s;
    a.rho = f->rho;
    a.v = f->v;
    a.feedback = (c->p.flags & RT_GAS_FEEDBACK) ? 1 : 0;
    a.T = f->T;
  }
  a.status = c->status;
  a.partials = c->partials;
  a.nparts = (int)ctx_step_blocks(c, true);
}

int ctx_init_host(const rt_grid *g, const rt_angles *an, const rt_params *p, rt_ctx *c) {
  if (!g || !an || !p) return RT_EINVAL;
  if (g->ndim < 1 || g->ndim > 3) return RT_EINVAL;
  long long nc = 1;
  for (int d = 0; d < 3; ++d) {
    if (g->n[d] < 1) return RT_EINVAL;
    if (d >= g->ndim && g->n[d] != 1) return RT_EINVAL;
    if (d < g->ndim) {
      if (!(g->dx[d] > 0.0) || !std::isfinite(g->dx[d])) return RT_EINVAL;
      for (int s = 0; s < 2; ++s)
        if (g->bc[d][s] < RT_BC_PERIODIC || g->bc[d][s] > RT_BC_VACUUM) return RT_EINVAL;
      if ((g->bc[d][0] == RT_BC_PERIODIC) != (g->bc[d][1] == RT_BC_PERIODIC)) return RT_EINVAL;
    }
    nc *= g->n[d];
  }
  if (nc > 0x7fffffffLL) return RT_EUNSUPPORTED;
  if (an->n < 1 || an->n > RT_MAX_ANGLES || !an->mu || !an->w) return RT_EINVAL;
  double wsum = 0.0;
  for (int m = 0; m < an->n; ++m) {
    const double *n = an->mu + 3 * m;
    const double nn = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    // 1D slabs may use azimuthally averaged directions (mu, 0, 0), |n| <= 1
    const bool norm_ok = g->ndim == 1 ? nn <= 1.0 + 1e-12 : std::fabs(nn - 1.0) <= 1e-12;
    if (!norm_ok || !(an->w[m] > 0.0)) return RT_EBADQUAD;
    wsum += an->w[m];
  }
  if (!(std::fabs(wsum - 1.0) <= 1e-12)) return RT_EBADQUAD;
  if (!(p->c > 0.0) || !(p->prat >= 0.0) || !(p->gamma > 1.0) || !(p->r_ideal > 0.0))
    return RT_EINVAL;
  if (p->precision != RT_FP64 && p->precision != RT_FP32_MIXED) return RT_EINVAL;
  if (!(p->c_reduced >= 0.0) || p->c_reduced > p->c) return RT_EINVAL;
  if (p->c_reduced > 0.0 && p->c_reduced < p->c && (p->flags & RT_ESTIMATE_V))
    return RT_EUNSUPPORTED;

  c->g = *g;
  c->p = *p;
  if (!(c->p.newton_rtol > 0.0)) c->p.newton_rtol = 1e-14;
  if (c->p.newton_maxit <= 0) c->p.newton_maxit = 64;
  c->nang = an->n;
  c->ncell = nc;
  c->all_periodic = true;
  for (int d = 0; d < g->ndim; ++d)
    if (g->bc[d][0] != RT_BC_PERIODIC) c->all_periodic = false;
  const int N = an->n;
  c->h_mu.assign(3 * (size_t)N, 0.0);
  c->h_w.assign(an->w, an->w + N);
  c->h_ghost.assign(6 * (size_t)N, 0.0);
  c->cfl_sum = 0.0;
  for (int m = 0; m < N; ++m) {
    double s = 0.0;
    for (int k = 0; k < 3; ++k) {
      c->h_mu[(size_t)k * N + m] = an->mu[3 * m + k];
      if (k < g->ndim) s += std::fabs(an->mu[3 * m + k]) / g->dx[k];
    }
    if (s > c->cfl_sum) c->cfl_sum = s;
  }
  c->shape = pick_shape(N, c->all_periodic, p->precision);
  // second order: the fused step runs both absorption solves on the
  // wave-group kernel; the step from a given dF on the thread-per-cell one
  if (p->flags & RT_SECOND_ORDER) c->shape.second = true;
  c->nblocks = (nc + 63) / 64;  // enough partial-total rows for either kernel
  // angle records: every slot of the wave-group kernel has one (padding
  // slots a zero record)
  const int slots = c->shape.waves * c->shape.groups * kAnglesPerWave;
  c->nrec = slots > N ? slots : N;
  return RT_OK;
}

namespace {
// Scratch layout: offsets of the pieces in one block.
struct Plan {
  size_t mu, w, muf, wf, ghost, arec, arecf, mom0, mom1, faces, partials, status, total;
};
Plan plan_of(const rt_ctx *c) {
  Plan q;
  const size_t N = c->nang, nc = c->ncell;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align256(bytes);
    return at;
  };
  q.mu = take(sizeof(double) * 3 * N);
  q.w = take(sizeof(double) * N);
  q.muf = take(sizeof(float) * 3 * N);
  q.wf = take(sizeof(float) * N);
  q.ghost = take(sizeof(double) * 6 * N);
  q.arec = take(sizeof(double) * kRec * (size_t)c->nrec);
  q.arecf = take(sizeof(float) * kRec * (size_t)c->nrec);
  q.mom0 = take(sizeof(double) * kNmomX * nc);
  q.mom1 = take(sizeof(double) * kNmomX * nc);
  q.faces = take(sizeof(double) * 9 * nc);
  q.partials = take(sizeof(double) * kNtot * c->nblocks);
  q.status = take(sizeof(int));
  q.total = o;
  return q;
}
}  // namespace

size_t ctx_scratch_bytes(const rt_ctx *c) { return plan_of(c).total; }

int ctx_attach_scratch(rt_ctx *c, char *base, hipStream_t s) {
  const Plan q = plan_of(c);
  const size_t N = c->nang;
  c->d_mu = reinterpret_cast<double *>(base + q.mu);
  c->d_w = reinterpret_cast<double *>(base + q.w);
  c->d_muf = reinterpret_cast<float *>(base + q.muf);
  c->d_wf = reinterpret_cast<float *>(base + q.wf);
  c->h_muf.assign(c->h_mu.begin(), c->h_mu.end());
  c->h_wf.assign(c->h_w.begin(), c->h_w.end());
  c->d_ghost = reinterpret_cast<double *>(base + q.ghost);
  c->d_arec = reinterpret_cast<double *>(base + q.arec);
  c->d_arecf = reinterpret_cast<float *>(base + q.arecf);
  c->mom[0] = reinterpret_cast<double *>(base + q.mom0);
  c->mom[1] = reinterpret_cast<double *>(base + q.mom1);
  c->faces = reinterpret_cast<double *>(base + q.faces);
  c->partials = reinterpret_cast<double *>(base + q.partials);
  c->status = reinterpret_cast<int *>(base + q.status);
  const bool ok =
      hip_ok(hipMemcpyAsync(c->d_mu, c->h_mu.data(), sizeof(double) * 3 * N,
                            hipMemcpyHostToDevice, s)) &&
      hip_ok(hipMemcpyAsync(c->d_w, c->h_w.data(), sizeof(double) * N, hipMemcpyHostToDevice,
                            s)) &&
      hip_ok(hipMemcpyAsync(c->d_muf, c->h_muf.data(), sizeof(float) * 3 * N,
                            hipMemcpyHostToDevice, s)) &&
      hip_ok(hipMemcpyAsync(c->d_wf, c->h_wf.data(), sizeof(float) * N, hipMemcpyHostToDevice,
                            s)) &&
      hip_ok(hipMemcpyAsync(c->d_ghost, c->h_ghost.data(), sizeof(double) * 6 * N,
                            hipMemcpyHostToDevice, s));
  if (!ok) return RT_EDEVICE;
  clear_stale_error();
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, s, c->status, 0);
  return hip_ok(hipGetLastError()) ? RT_OK : RT_EDEVICE;
}

int ctx_moments(rt_ctx *c, hipStream_t s) {
  StepArgs a;
  ctx_fill_args(c, 1.0, nullptr, a);
  a.I_in = c->I[c->cur];
  a.mom_out = c->mom[c->mom_cur];
  launch_moments(c, a, s);
  if (!hip_ok(hipGetLastError())) return RT_EDEVICE;
  c->mom_valid = true;
  return RT_OK;
}

// Per-call tables: interface alpha / flow speed / IV Courant factor for this
// dt and fields, and 3 v J of the current moments.
int ctx_prepare_call(rt_ctx *c, double dt, const rt_fields *f, hipStream_t s) {
  StepArgs a;
  ctx_fill_args(c, dt, f, a);
  clear_stale_error();
  const long long nthreads = c->ncell > c->nrec ? c->ncell : c->nrec;
  hipLaunchKernelGGL(k_faces, dim3((unsigned)((nthreads + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     s, a, c->faces, c->mom[c->mom_cur], c->d_arec, c->d_arecf, c->nrec);
  return hip_ok(hipGetLastError()) ? RT_OK : RT_EDEVICE;
}

int ctx_step(rt_ctx *c, double dt, int nsteps, const rt_fields *f, rt_out *o, hipStream_t s) {
  int st = ensure_moments(c, s);
  if (st != RT_OK) return st;
  st = ctx_prepare_call(c, dt, f, s);
  if (st != RT_OK) return st;
  return ctx_step_range(c, dt, f, o, 0, nsteps, nsteps, s);
}

int ctx_step_range(rt_ctx *c, double dt, const rt_fields *f, rt_out *o, int k0, int k1,
                   int ntotal, hipStream_t s) {
  const bool feedback = (c->p.flags & RT_GAS_FEEDBACK) != 0;
  for (int k = k0; k < k1; ++k) {
    // with gas feedback the flow speeds of the interface table follow v
    if (feedback && k > k0) {
      const int st = ctx_prepare_call(c, dt, f, s);
      if (st != RT_OK) return st;
    }
    const int st = one_step(c, dt, f, nullptr, true, o, k == 0, k == ntotal - 1, s);
    if (st != RT_OK) return st;
  }
  return RT_OK;
}

int ctx_init_equilibrium(rt_ctx *c, const double *T, void *I, hipStream_t s) {
  dim3 g((unsigned)cell_blocks(c)), b(kBlock);
  clear_stale_error();
  if (c->p.precision == RT_FP32_MIXED)
    hipLaunchKernelGGL(k_equilibrium<float>, g, b, 0, s, T, static_cast<float *>(I),
                       (int)c->ncell, c->nang);
  else
    hipLaunchKernelGGL(k_equilibrium<double>, g, b, 0, s, T, static_cast<double *>(I),
                       (int)c->ncell, c->nang);
  return hip_ok(hipGetLastError()) ? RT_OK : RT_EDEVICE;
}

}  // namespace rtk

// ------------------------------------------------------ static scratch
// The library scratch of rt_step_static: one array per GPU (each device that
// runs the library holds its own copy until the process ends).  Host code
// reaches it only through the device address that hipGetSymbolAddress gives
// for the current device, once per device, kept in static_ptr[]; the array's
// name is a host-side stand-in, not a device address.
static __device__ __align__(256) char scratch[RT_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kStaticDevices = 16;
std::mutex static_mu;
char *static_ptr[kStaticDevices];
// Host contexts of rt_step_static, one per device, with their host tables
// reserved for RT_MAX_ANGLES directions when the library loads, so that the
// calls themselves allocate nothing (the tables are refilled in place).
rt_ctx *static_ctx[kStaticDevices];

__attribute__((constructor)) void static_ctx_init() {
  for (int d = 0; d < kStaticDevices; ++d) {
    rt_ctx *c = new (std::nothrow) rt_ctx();
    if (!c) continue;
    const size_t N = RT_MAX_ANGLES;
    c->h_mu.reserve(3 * N);
    c->h_w.reserve(N);
    c->h_ghost.reserve(6 * N);
    c->h_muf.reserve(3 * N);
    c->h_wf.reserve(N);
    static_ctx[d] = c;
  }
}
}  // namespace

using namespace rtk;

extern "C" {

int rt_step_static(const rt_grid *g, const rt_angles *an, const rt_params *p, void *Ia, void *Ib,
                   double dt, int nsteps, const rt_fields *f, rt_out *o, int *status,
                   void *stream) {
  if (!g || !an || !p || !Ia || !Ib || Ia == Ib || !fields_ok(f) || !status || nsteps < 0)
    return RT_EINVAL;
  int dev = -1;
  if (!hip_ok(hipGetDevice(&dev)) || dev < 0 || dev >= kStaticDevices) return RT_EDEVICE;
  char *base = nullptr;
  {
    std::lock_guard<std::mutex> lk(static_mu);
    if (!static_ptr[dev]) {
      void *ptr = nullptr;
      if (!hip_ok(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch))) || !ptr) {
        clear_stale_error();
        return RT_EDEVICE;
      }
      static_ptr[dev] = static_cast<char *>(ptr);
    }
    base = static_ptr[dev];
  }
  rt_ctx *c = static_ctx[dev];
  if (!c) return RT_ENOMEM;
  c->owns_device = false;
  c->profile = false;
  for (auto &t : c->d_gface) t = nullptr;
  int st = ctx_init_host(g, an, p, c);
  if (st != RT_OK) return st;
  if (ctx_scratch_bytes(c) > RT_STATIC_SCRATCH_BYTES) return RT_ETOOBIG;
  if ((c->p.flags & RT_GAS_FEEDBACK) && !c->shape.waves) return RT_EUNSUPPORTED;
  st = ctx_check_dt(c, dt);
  if (st != RT_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  st = ctx_attach_scratch(c, base, s);
  if (st != RT_OK) return st;
  c->status = status;  // the caller's flag
  c->I[0] = Ia;
  c->I[1] = Ib;
  c->cur = 0;
  c->mom_cur = 0;
  c->mom_valid = false;
  return ctx_step(c, dt, nsteps, f, o, s);
}


const char *rt_strerror(int st) {
  switch (st) {
    case RT_OK: return "ok";
    case RT_PENDING: return "request still in flight";
    case RT_EINVAL: return "invalid argument";
    case RT_ENOMEM: return "out of memory";
    case RT_EDEVICE: return "HIP runtime error";
    case RT_ECFL: return "time step violates the transport CFL limit";
    case RT_ENOCONV: return "temperature Newton iteration failed";
    case RT_EBADQUAD: return "invalid angle set (weights or direction norms)";
    case RT_ESTATE: return "call order violated (no intensity bound?)";
    case RT_EUNSUPPORTED: return "unsupported request";
    case RT_ETOOBIG: return "problem scratch exceeds the static scratch array";
    default: return "unknown status";
  }
}

int rt_create(const rt_grid *g, const rt_angles *an, const rt_params *p, rt_ctx **out) {
  if (!out) return RT_EINVAL;
  *out = nullptr;
  rt_ctx *c = new (std::nothrow) rt_ctx();
  if (!c) return RT_ENOMEM;
  int st = ctx_init_host(g, an, p, c);
  if (st != RT_OK) {
    delete c;
    return st;
  }
  hipGetDevice(&c->device);
  char *base = nullptr;
  if (!hip_ok(hipMalloc(&base, ctx_scratch_bytes(c)))) {
    delete c;
    return RT_ENOMEM;
  }
  c->owns_device = true;
  st = ctx_attach_scratch(c, base, nullptr);
  if (st == RT_OK && !hip_ok(hipStreamSynchronize(nullptr))) st = RT_EDEVICE;
  if (st != RT_OK) {
    rt_destroy(c);
    return st;
  }
  *out = c;
  return RT_OK;
}

int rt_destroy(rt_ctx *c) {
  if (!c) return RT_EINVAL;
  hipDeviceSynchronize();
  // the scratch block starts at the angle table
  if (c->owns_device && c->d_mu) hipFree(c->d_mu);
  for (auto f : c->d_gface)
    if (f) hipFree(f);
  for (auto &pr : c->pending) {
    hipEventDestroy(pr.first);
    hipEventDestroy(pr.second);
  }
  for (auto e : c->ev_pool) hipEventDestroy(e);
  delete c;
  return RT_OK;
}

int rt_bind_intensity(rt_ctx *c, void *Ia, void *Ib) {
  if (!c || !Ia || !Ib || Ia == Ib) return RT_EINVAL;
  c->I[0] = Ia;
  c->I[1] = Ib;
  c->cur = 0;
  c->mom_valid = false;
  return RT_OK;
}

int rt_current_intensity(rt_ctx *c, void **cur) {
  if (!c || !cur) return RT_EINVAL;
  if (!c->I[0]) return RT_ESTATE;
  *cur = c->I[c->cur];
  return RT_OK;
}

int rt_set_fixed_bc(rt_ctx *c, int axis, int side, const double *tab) {
  if (!c || !tab || axis < 0 || axis >= c->g.ndim || side < 0 || side > 1) return RT_EINVAL;
  if (c->g.bc[axis][side] != RT_BC_FIXED) return RT_EINVAL;
  const int f = axis * 2 + side;
  const size_t off = (size_t)f * c->nang;
  std::memcpy(&c->h_ghost[off], tab, sizeof(double) * c->nang);
  // steps queued on a caller's stream may still read the table: the upload
  // waits for them (the null-stream copy alone does not order against
  // non-blocking streams)
  if (!hip_ok(hipDeviceSynchronize())) return RT_EDEVICE;
  if (!hip_ok(hipMemcpy(c->d_ghost + off, tab, sizeof(double) * c->nang, hipMemcpyHostToDevice)))
    return RT_EDEVICE;
  // the angle table replaces a position-dependent one
  if (c->d_gface[f]) {
    hipFree(c->d_gface[f]);
    c->d_gface[f] = nullptr;
  }
  return RT_OK;
}

int rt_set_fixed_bc_face(rt_ctx *c, int axis, int side, const double *tab) {
  if (!c || !tab || axis < 0 || axis >= c->g.ndim || side < 0 || side > 1) return RT_EINVAL;
  if (c->g.bc[axis][side] != RT_BC_FIXED || !c->owns_device) return RT_EINVAL;
  const int f = axis * 2 + side;
  const size_t n = (size_t)c->nang * (size_t)(c->ncell / c->g.n[axis]);
  if (!c->d_gface[f]) {
    if (hipMalloc(&c->d_gface[f], sizeof(double) * n) != hipSuccess) {
      c->d_gface[f] = nullptr;
      clear_stale_error();
      return RT_ENOMEM;
    }
  } else {
    hipDeviceSynchronize();  // a step in flight may still read the table
  }
  if (!hip_ok(hipMemcpy(c->d_gface[f], tab, sizeof(double) * n, hipMemcpyHostToDevice)))
    return RT_EDEVICE;
  return RT_OK;
}

int rt_moments(rt_ctx *c, rt_out *o, void *stream) {
  if (!c) return RT_EINVAL;
  if (!c->I[0]) return RT_ESTATE;
  hipStream_t s = (hipStream_t)stream;
  StepArgs a;
  ctx_fill_args(c, 1.0, nullptr, a);
  a.I_in = c->I[c->cur];
  a.mom_out = c->mom[c->mom_cur];
  if (o) {
    a.oE = o->Er;
    a.oF = o->Fr;
    a.oP = o->Pr;
  }
  launch_moments(c, a, s);
  if (!hip_ok(hipGetLastError())) return RT_EDEVICE;
  c->mom_valid = true;
  return RT_OK;
}

int rt_transport(rt_ctx *c, double dt, const rt_fields *f, void *dF, void *stream) {
  if (!c || !dF || !fields_ok(f)) return RT_EINVAL;
  if (!c->I[0]) return RT_ESTATE;
  int st = ctx_check_dt(c, dt);
  if (st != RT_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  st = ensure_moments(c, s);
  if (st != RT_OK) return st;
  st = ctx_prepare_call(c, dt, f, s);
  if (st != RT_OK) return st;
  StepArgs a;
  ctx_fill_args(c, dt, f, a);
  a.I_in = c->I[c->cur];
  a.mom_in = c->mom[c->mom_cur];
  a.dF_out = dF;
  launch_transport(c, a, s);
  return hip_ok(hipGetLastError()) ? RT_OK : RT_EDEVICE;
}

int rt_source_implicit(rt_ctx *c, double dt, const rt_fields *f, const void *dF, rt_out *o,
                       void *stream) {
  if (!c || !fields_ok(f)) return RT_EINVAL;
  if (!c->I[0]) return RT_ESTATE;
  if ((c->p.flags & RT_GAS_FEEDBACK) && !c->shape.waves) return RT_EUNSUPPORTED;
  // the second-order step from a given dF runs per cell, without feedback
  if ((c->p.flags & RT_GAS_FEEDBACK) && c->shape.second) return RT_EUNSUPPORTED;
  if (!(dt > 0.0) || !std::isfinite(dt)) return RT_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  int st = ensure_moments(c, s);
  if (st != RT_OK) return st;
  st = ctx_prepare_call(c, dt, f, s);
  if (st != RT_OK) return st;
  return one_step(c, dt, f, dF, false, o, true, true, s);
}

int rt_step(rt_ctx *c, double dt, int nsteps, const rt_fields *f, rt_out *o, void *stream) {
  if (!c || !fields_ok(f) || nsteps < 0) return RT_EINVAL;
  if (!c->I[0]) return RT_ESTATE;
  if ((c->p.flags & RT_GAS_FEEDBACK) && !c->shape.waves) return RT_EUNSUPPORTED;
  int st = ctx_check_dt(c, dt);
  if (st != RT_OK) return st;
  return ctx_step(c, dt, nsteps, f, o, (hipStream_t)stream);
}

int rt_equilibrium_intensity(rt_ctx *c, const double *T, void *I, void *stream) {
  if (!c || !T || !I) return RT_EINVAL;
  if (I == c->I[c->cur]) c->mom_valid = false;
  return ctx_init_equilibrium(c, T, I, (hipStream_t)stream);
}

int rt_sync_status(rt_ctx *c) {
  if (!c) return RT_EINVAL;
  if (!hip_ok(hipDeviceSynchronize())) return RT_EDEVICE;
  int h = 0;
  if (!hip_ok(hipMemcpy(&h, c->status, sizeof(int), hipMemcpyDeviceToHost))) return RT_EDEVICE;
  if (h) {
    hipMemset(c->status, 0, sizeof(int));
    return RT_ENOCONV;
  }
  return RT_OK;
}

int rt_profile_enable(rt_ctx *c, int enable) {
  if (!c) return RT_EINVAL;
  c->profile = enable != 0;
  return RT_OK;
}

int rt_profile_read(rt_ctx *c, double *total_ms, int *launches) {
  if (!c) return RT_EINVAL;
  for (auto &pr : c->pending) {
    if (!hip_ok(hipEventSynchronize(pr.second))) return RT_EDEVICE;
    float ms = 0.f;
    if (!hip_ok(hipEventElapsedTime(&ms, pr.first, pr.second))) return RT_EDEVICE;
    c->prof_ms += ms;
    c->prof_n += 1;
    c->ev_pool.push_back(pr.first);
    c->ev_pool.push_back(pr.second);
  }
  c->pending.clear();
  if (total_ms) *total_ms = c->prof_ms;
  if (launches) *launches = c->prof_n;
  c->prof_ms = 0.0;
  c->prof_n = 0;
  return RT_OK;
}

int rt_get_info(rt_ctx *c, rt_info *info) {
  if (!c || !info) return RT_EINVAL;
  info->nang = c->nang;
  info->ncell = c->ncell;
  info->storage_bytes = ctx_storage_bytes(c);
  info->block_threads = c->shape.waves ? 64 * c->shape.waves : kBlock;
  info->grid_blocks = ctx_step_blocks(c, true);
  return RT_OK;
}

}  // extern "C"
