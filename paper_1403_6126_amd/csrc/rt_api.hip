// Host side of the C ABI declared in include/rt.h: context management,
// validation, and the launches of the step kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "rt.h"
#include "rt_fallback.hpp"
#include "rt_step3.hpp"

using namespace rtk;

struct rt_ctx {
  rt_grid g;
  rt_params p;
  int nang;
  long long ncell;
  int device;
  bool all_periodic;
  double cfl_sum;  // max over angles of sum_d |mu_d| / dx_d
  std::vector<double> h_mu, h_w, h_ghost;
  double *d_mu = nullptr, *d_w = nullptr, *d_ghost = nullptr;
  void *I[2] = {nullptr, nullptr};
  int cur = 0;
  double *mom[2] = {nullptr, nullptr};  // [13][ncell]: E, F, P, 3vJ
  int mom_cur = 0;
  double *faces = nullptr;              // [3][3][ncell] interface table of the call
  int waves = 0;                        // waves per block of k_step3 (0: thread-per-cell kernel)
  bool mom_valid = false;
  double *partials = nullptr;
  double *acc = nullptr;
  int *status = nullptr;
  long long nblocks = 0;
  bool profile = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
  double prof_ms = 0.0;
  int prof_n = 0;
};

namespace {

bool hip_ok(hipError_t e) { return e == hipSuccess; }

int storage_bytes(const rt_ctx *c) { return c->p.precision == RT_FP32_MIXED ? 4 : 8; }

void fill_args(const rt_ctx *c, double dt, const rt_fields *f, StepArgs &a) {
  std::memset(&a, 0, sizeof(a));
  a.ndim = c->g.ndim;
  for (int d = 0; d < 3; ++d) {
    a.n[d] = c->g.n[d];
    for (int s = 0; s < 2; ++s) a.bc[d][s] = c->g.bc[d][s];
    a.dt_dx[d] = dt / c->g.dx[d];
    a.dl10[d] = 10.0 * c->g.dx[d];
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
  a.cvfac = c->p.r_ideal / (c->p.gamma - 1.0);
  double vol = 1.0;
  for (int d = 0; d < c->g.ndim; ++d) vol *= c->g.dx[d];
  a.vol = vol;
  a.rtol = c->p.newton_rtol;
  a.maxit = c->p.newton_maxit;
  a.estimate_v = (c->p.flags & RT_ESTIMATE_V) ? 1 : 0;
  a.mu = c->d_mu;
  a.w = c->d_w;
  a.ghost = c->d_ghost;
  a.faces = c->faces;
  if (f) {
    a.sa = f->sigma_a;
    a.ss = f->sigma_s;
    a.rho = f->rho;
    a.v = f->v;
    a.T = f->T;
  }
  a.status = c->status;
  a.partials = c->partials;
}

bool fields_ok(const rt_fields *f) {
  return f && f->sigma_a && f->sigma_s && f->rho && f->T && f->v;
}

int check_dt(const rt_ctx *c, double dt) {
  if (!(dt > 0.0) || !std::isfinite(dt)) return RT_EINVAL;
  if (c->p.c * dt * c->cfl_sum > 1.0 + 1e-12) return RT_ECFL;
  return RT_OK;
}

// Waves per block of the wave-group kernel (10 angles per wave), or 0 when
// the angle set is larger than it handles and the thread-per-cell kernel
// runs instead.
constexpr int kAnglesPerWave = 10;
int pick_waves(int nang) {
  const int G = (nang + kAnglesPerWave - 1) / kAnglesPerWave;
  return G <= kMaxWaves ? G : 0;
}

long long step_blocks(const rt_ctx *c) {
  return c->waves ? (c->ncell + 63) / 64 : (c->ncell + kBlock - 1) / kBlock;
}
long long cell_blocks(const rt_ctx *c) { return (c->ncell + kBlock - 1) / kBlock; }

template <typename S, typename A, bool FUSED>
void launch_step_t(const rt_ctx *c, const StepArgs &a, hipStream_t s) {
  if (c->waves) {
    dim3 g((unsigned)step_blocks(c)), b(64 * c->waves);
    if (c->all_periodic)
      hipLaunchKernelGGL((k_step3<S, A, kAnglesPerWave, true, FUSED>), g, b, 0, s, a);
    else
      hipLaunchKernelGGL((k_step3<S, A, kAnglesPerWave, false, FUSED>), g, b, 0, s, a);
  } else {
    dim3 g((unsigned)step_blocks(c)), b(kBlock);
    if (c->all_periodic)
      hipLaunchKernelGGL((k_step<S, A, true, FUSED>), g, b, 0, s, a);
    else
      hipLaunchKernelGGL((k_step<S, A, false, FUSED>), g, b, 0, s, a);
  }
}

void launch_step(const rt_ctx *c, const StepArgs &a, bool fused, hipStream_t s) {
  if (c->p.precision == RT_FP32_MIXED) {
    if (fused)
      launch_step_t<float, float, true>(c, a, s);
    else
      launch_step_t<float, float, false>(c, a, s);
  } else {
    if (fused)
      launch_step_t<double, double, true>(c, a, s);
    else
      launch_step_t<double, double, false>(c, a, s);
  }
}

void launch_transport(const rt_ctx *c, const StepArgs &a, hipStream_t s) {
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
  dim3 g((unsigned)cell_blocks(c)), b(kBlock);
  if (c->p.precision == RT_FP32_MIXED)
    hipLaunchKernelGGL(k_moments<float>, g, b, 0, s, a);
  else
    hipLaunchKernelGGL(k_moments<double>, g, b, 0, s, a);
}

int ensure_moments(rt_ctx *c, hipStream_t s) {
  if (c->mom_valid) return RT_OK;
  StepArgs a;
  fill_args(c, 1.0, nullptr, a);
  a.I_in = c->I[c->cur];
  a.mom_out = c->mom[c->mom_cur];
  launch_moments(c, a, s);
  if (!hip_ok(hipGetLastError())) return RT_EDEVICE;
  c->mom_valid = true;
  return RT_OK;
}

// Per-call tables: interface alpha / flow speed / IV Courant factor for this
// dt and fields, and 3 v J of the current moments.
int prepare_call(rt_ctx *c, double dt, const rt_fields *f, hipStream_t s) {
  StepArgs a;
  fill_args(c, dt, f, a);
  const long long nb = (c->ncell + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_faces, dim3((unsigned)nb), dim3(kBlock), 0, s, a, c->faces,
                     c->mom[c->mom_cur]);
  return hip_ok(hipGetLastError()) ? RT_OK : RT_EDEVICE;
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
  fill_args(c, dt, f, a);
  a.I_in = c->I[c->cur];
  a.I_out = c->I[1 - c->cur];
  a.mom_in = c->mom[c->mom_cur];
  a.mom_out = c->mom[1 - c->mom_cur];
  a.dF_in = dF;
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
  hipLaunchKernelGGL(k_totals, dim3(1), dim3(kBlock), 0, s, c->partials, (int)step_blocks(c),
                     c->acc, first ? 1 : 0, (last && o) ? o->totals : nullptr);
  if (!hip_ok(hipGetLastError())) return RT_EDEVICE;
  c->cur = 1 - c->cur;
  c->mom_cur = 1 - c->mom_cur;
  c->mom_valid = true;
  return RT_OK;
}

}  // namespace

extern "C" {

const char *rt_strerror(int st) {
  switch (st) {
    case RT_OK: return "ok";
    case RT_EINVAL: return "invalid argument";
    case RT_ENOMEM: return "out of memory";
    case RT_EDEVICE: return "HIP runtime error";
    case RT_ECFL: return "time step violates the transport CFL limit";
    case RT_ENOCONV: return "temperature Newton iteration failed";
    case RT_EBADQUAD: return "invalid angle set (weights or direction norms)";
    case RT_ESTATE: return "call order violated (no intensity bound?)";
    case RT_EUNSUPPORTED: return "unsupported request";
    default: return "unknown status";
  }
}

int rt_create(const rt_grid *g, const rt_angles *an, const rt_params *p, rt_ctx **out) {
  if (!out) return RT_EINVAL;
  *out = nullptr;
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

  rt_ctx *c = new (std::nothrow) rt_ctx();
  if (!c) return RT_ENOMEM;
  c->g = *g;
  c->p = *p;
  if (!(c->p.newton_rtol > 0.0)) c->p.newton_rtol = 1e-14;
  if (c->p.newton_maxit <= 0) c->p.newton_maxit = 64;
  c->nang = an->n;
  c->ncell = nc;
  hipGetDevice(&c->device);
  c->all_periodic = true;
  for (int d = 0; d < g->ndim; ++d)
    if (g->bc[d][0] != RT_BC_PERIODIC) c->all_periodic = false;
  const int N = an->n;
  c->h_mu.assign(3 * N, 0.0);
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
  c->waves = pick_waves(N);
  c->nblocks = (nc + 63) / 64;  // enough partial-total rows for either kernel
  bool ok = hip_ok(hipMalloc(&c->d_mu, sizeof(double) * 3 * N)) &&
            hip_ok(hipMalloc(&c->d_w, sizeof(double) * N)) &&
            hip_ok(hipMalloc(&c->d_ghost, sizeof(double) * 6 * N)) &&
            hip_ok(hipMalloc(&c->mom[0], sizeof(double) * kNmomX * nc)) &&
            hip_ok(hipMalloc(&c->mom[1], sizeof(double) * kNmomX * nc)) &&
            hip_ok(hipMalloc(&c->faces, sizeof(double) * 9 * nc)) &&
            hip_ok(hipMalloc(&c->partials, sizeof(double) * kNtot * c->nblocks)) &&
            hip_ok(hipMalloc(&c->acc, sizeof(double) * kNtot)) &&
            hip_ok(hipMalloc(&c->status, sizeof(int)));
  if (ok)
    ok = hip_ok(hipMemcpy(c->d_mu, c->h_mu.data(), sizeof(double) * 3 * N,
                          hipMemcpyHostToDevice)) &&
         hip_ok(hipMemcpy(c->d_w, c->h_w.data(), sizeof(double) * N, hipMemcpyHostToDevice)) &&
         hip_ok(hipMemcpy(c->d_ghost, c->h_ghost.data(), sizeof(double) * 6 * N,
                          hipMemcpyHostToDevice)) &&
         hip_ok(hipMemset(c->status, 0, sizeof(int))) &&
         hip_ok(hipMemset(c->acc, 0, sizeof(double) * kNtot));
  if (!ok) {
    rt_destroy(c);
    return RT_ENOMEM;
  }
  *out = c;
  return RT_OK;
}

int rt_destroy(rt_ctx *c) {
  if (!c) return RT_EINVAL;
  hipDeviceSynchronize();
  hipFree(c->d_mu);
  hipFree(c->d_w);
  hipFree(c->d_ghost);
  hipFree(c->mom[0]);
  hipFree(c->mom[1]);
  hipFree(c->faces);
  hipFree(c->partials);
  hipFree(c->acc);
  hipFree(c->status);
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
  const size_t off = (size_t)(axis * 2 + side) * c->nang;
  std::memcpy(&c->h_ghost[off], tab, sizeof(double) * c->nang);
  if (!hip_ok(hipMemcpy(c->d_ghost + off, tab, sizeof(double) * c->nang, hipMemcpyHostToDevice)))
    return RT_EDEVICE;
  return RT_OK;
}

int rt_moments(rt_ctx *c, rt_out *o, void *stream) {
  if (!c) return RT_EINVAL;
  if (!c->I[0]) return RT_ESTATE;
  hipStream_t s = (hipStream_t)stream;
  StepArgs a;
  fill_args(c, 1.0, nullptr, a);
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
  int st = check_dt(c, dt);
  if (st != RT_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  st = ensure_moments(c, s);
  if (st != RT_OK) return st;
  st = prepare_call(c, dt, f, s);
  if (st != RT_OK) return st;
  StepArgs a;
  fill_args(c, dt, f, a);
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
  if (!(dt > 0.0) || !std::isfinite(dt)) return RT_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  int st = ensure_moments(c, s);
  if (st != RT_OK) return st;
  st = prepare_call(c, dt, f, s);
  if (st != RT_OK) return st;
  return one_step(c, dt, f, dF, false, o, true, true, s);
}

int rt_step(rt_ctx *c, double dt, int nsteps, const rt_fields *f, rt_out *o, void *stream) {
  if (!c || !fields_ok(f) || nsteps < 0) return RT_EINVAL;
  if (!c->I[0]) return RT_ESTATE;
  int st = check_dt(c, dt);
  if (st != RT_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  st = ensure_moments(c, s);
  if (st != RT_OK) return st;
  st = prepare_call(c, dt, f, s);
  if (st != RT_OK) return st;
  for (int k = 0; k < nsteps; ++k) {
    st = one_step(c, dt, f, nullptr, true, o, k == 0, k == nsteps - 1, s);
    if (st != RT_OK) return st;
  }
  return RT_OK;
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
  info->storage_bytes = storage_bytes(c);
  info->block_threads = c->waves ? 64 * c->waves : kBlock;
  info->grid_blocks = step_blocks(c);
  return RT_OK;
}

}  // extern "C"
