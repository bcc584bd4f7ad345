// Fused step kernel with the waves of a block sharing cells (angle-major
// layout I[m][c]).
//
// A block holds 64 consecutive cells (one per lane) and G <= 8 waves; the
// angles are cut into groups of KA, and wave g owns the groups g, g + G, ...
// (NG of them at most, so up to NG*G*KA angles).  Within a wave the angle is
// uniform, so the direction cosines, weights and the upwind
// direction of every axis are scalars, and every intensity load reads 64
// consecutive cells of one angle plane.  Per step:
//   axes     the stencil data of each active axis (cell indices, ghost
//            kinds, 3vJ differences, face coefficients) built by one wave
//            and shared with the others through LDS;
//   phase A  transport increment of the wave's angles (Section 4.2), one
//            active axis at a time: the flux difference of the two faces
//            from the differences of I~ and IV between consecutive stencil
//            cells, with a per-call interface table (C alpha, IV upwinding)
//            and per-angle records (mu_d, 1 - nu, weights) read as scalars;
//   phase B  the absorption right-hand side r4 and the wave's partial sums of
//            the per-cell sums of the reduced absorption and scattering
//            systems; the per-angle values stay in registers;
//   reduce   the partial sums across the waves (LDS, fixed order);
//   solve    FP64 Newton on the quartic in T' and the 2 x 2 scattering
//            system, on every wave or on wave 0 with the solution passed on
//            through LDS;
//   phase C  I^{n+1} of the wave's angles, written once, and the partial
//            moments, reduced across the waves like the sums.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rt_common.hpp"
#include "rt_internal.hpp"

namespace rtk {

constexpr int kNsum = 22;        // per-cell sums of phase B
constexpr int kChunk = 11;       // values reduced per LDS round

// Half the van Leer harmonic-mean slope of two consecutive differences:
// ab/(a + b) when ab > 0, else 0 (zero at extrema).  The upwind interface
// value of the monotonic piecewise-linear reconstruction at Courant number
// nu is the upwind cell's value plus (1 - nu) times this, signed by the
// direction.  It is symmetric in a and b, and odd under a, b -> -a, -b.
template <typename A>
__device__ __forceinline__ A vl_half(A a, A b) {
  const A ab = a * b;
  const A q = ab * limiter_rcp(a + b);
  return ab > A(0) ? q : A(0);
}

// Transport data of one cell along one axis, shared by every angle slot of
// the wave (loaded once per axis).
//
// The flux difference of a cell needs the intensities of the cells -2..+2
// only through their consecutive differences: with D_k the differences of
// I~ = I - IV/C between cells -2|-1, -1|0, 0|+1, +1|+2 (k = 0..3), the
// alpha-blend of the two faces (Section 4.2) gives, for mu_d > 0,
//   x_R - x_L = Cb_R D_2 + (Ca_L + Cb_L) D_1 + h2 (Ca_R q_0 - Ca_L q_-1),
// and for mu_d < 0
//   x_R - x_L = (Ca_R + Cb_R) D_2 + Cb_L D_1 - h2 (Ca_R q_+1 - Ca_L q_0),
// Ca = C alpha, Cb = C (1 - alpha)/2, h2 = 1 - nu, q the half slopes of
// I~; the cell's own C I~ cancels between the faces (Ca + 2 Cb = C).  The
// IV values of the two faces likewise differ by
//   (1 - l_R) V_2 + l_L V_1 + f_R qv_R - f_L qv_L,
// V_k the differences of IV = n.W (W = 3 v J) and qv the half slope of the
// face's upwind cell.
template <typename A>
struct AxisData {
  unsigned idx[4];  // cells at offsets -2, -1, +1, +2 (wrapped, or the edge cell)
  int kind[4];      // 0 read the cell, 1 fixed table, 2 vacuum
  A dW[4][3];       // W(-1)-W(-2), W(0)-W(-1), W(+1)-W(0), W(+2)-W(+1)
  A caL, cbL, caR, cbR;
  A lL, rR;         // l of the low face, 1 - l of the high face
  A fL, fR;         // signed IV slope factors of the two faces
};

template <typename A, bool PER>
__device__ __forceinline__ void load_axis(const StepArgs &p, int c, const int q[3], int d,
                                          const A (&Wc)[3], AxisData<A> &s) {
  const int n = p.n[d];
  const size_t N = (size_t)p.ncell;
  const int offs[4] = {-2, -1, 1, 2};
  A W[4][3];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int k = q[d] + offs[j];
    int kk = k, kind = 0;
    if (k < 0 || k >= n) {
      const int bc = PER ? kPeriodic : p.bc[d][k < 0 ? 0 : 1];
      if (bc == kPeriodic) {
        kk = ((k % n) + n) % n;
      } else {
        kk = k < 0 ? 0 : n - 1;
        kind = bc == kFixed ? 1 : bc == kVacuum ? 2 : 0;
      }
    }
    const int cj = c + (kk - q[d]) * p.stride[d];
    s.idx[j] = (unsigned)cj;
    s.kind[j] = kind;
#pragma unroll
    for (int t = 0; t < 3; ++t) W[j][t] = A(p.mom_in[(size_t)(10 + t) * N + cj]);
  }
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    s.dW[0][t] = W[1][t] - W[0][t];
    s.dW[1][t] = Wc[t] - W[1][t];
    s.dW[2][t] = W[2][t] - Wc[t];
    s.dW[3][t] = W[3][t] - W[2][t];
  }
  const A hC = A(0.5 * p.C);
  s.caL = A(p.faces[(size_t)(d * 3 + 0) * N + c]);
  s.lL = A(p.faces[(size_t)(d * 3 + 1) * N + c]);
  s.fL = A(p.faces[(size_t)(d * 3 + 2) * N + c]);
  if (PER || q[d] + 1 < n || p.bc[d][1] == kPeriodic) {
    const unsigned cr = s.idx[2];
    s.caR = A(p.faces[(size_t)(d * 3 + 0) * N + cr]);
    s.rR = A(1.0 - p.faces[(size_t)(d * 3 + 1) * N + cr]);
    s.fR = A(p.faces[(size_t)(d * 3 + 2) * N + cr]);
  } else {
    // high non-periodic boundary: the ghost copies this cell's fields
    const double u = p.v[(size_t)d * N + c];
    s.caR = A(p.C * alpha_of(p.sa[c] + p.ss[c], p.dl10[d]));
    s.rR = A(1.0 - iv_lower_share(u));
    s.fR = A(iv_signed_factor(u, p.dt_dx[d]));
  }
  s.cbL = hC - A(0.5) * s.caL;
  s.cbR = hC - A(0.5) * s.caR;
  // dt/dx_d taken into the face coefficients: the increment is then
  // -mu_d times the sum they weight
  const A dtdx = A(p.dt_dx[d]);
  s.caL *= dtdx;
  s.cbL *= dtdx;
  s.caR *= dtdx;
  s.cbR *= dtdx;
  s.lL *= dtdx;
  s.rR *= dtdx;
  s.fL *= dtdx;
  s.fR *= dtdx;
}

// Element idx of an angle plane, addressed by a 32-bit byte offset from the
// wave-uniform start of the plane (one scalar base and one vector register
// per load).  rt_create keeps every plane below 4 GiB.
template <typename S>
__device__ __forceinline__ S plane_ld(const S *plane, unsigned idx) {
  const unsigned off = idx * (unsigned)sizeof(S);
  return *reinterpret_cast<const S *>(reinterpret_cast<const char *>(plane) + off);
}

// The same read as a raw buffer load: the plane is a buffer resource held in
// scalar registers, the lane's byte offset one vector register, so no vector
// address arithmetic is needed (gfx9 resource word 3 for raw loads).
template <typename S>
__device__ __forceinline__ S plane_buf_ld(const S *plane, unsigned idx) {
  const __amdgpu_buffer_rsrc_t r =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<S *>(plane), 0, 0x7fffffff, 0x00020000);
  const unsigned off = idx * (unsigned)sizeof(S);
  if constexpr (sizeof(S) == 8)
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
  else
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

// Intensity at a stencil cell from the value raw read at its (clamped) cell
// idx of the angle plane, with the ghost kinds.  ghosts (wave-uniform): some
// lane of the wave has a ghost cell along this axis; without any, the
// per-lane kind tests are skipped by a scalar branch.
template <typename S, typename A, bool PER>
__device__ __forceinline__ A plane_value(const StepArgs &p, S raw, int idx, int kind, int side,
                                         int d, int m, A mud, bool ghosts) {
  if (PER || !ghosts) return A(raw);
  if (kind == 0) return A(raw);
  if (kind == 1) return A(fixed_ghost(p, d, side, m, idx));
  const bool outgoing = side == 0 ? (mud < A(0)) : (mud > A(0));
  return outgoing ? A(raw) : A(0);
}

// Sum (or, for the last value when MINLAST, minimum) of NV values over the
// G waves of the block, lane by lane, in a fixed order, R values per LDS
// round; every wave receives the totals.  The rounds only bound the LDS
// footprint (buf: G*R*64, tot: R*64 doubles): the result is the same for
// every R.
template <int NV, bool MINLAST, int R>
__device__ __forceinline__ void waves_reduce(double (&x)[NV], double *buf, double *tot, int g,
                                             int G, int lane) {
#pragma unroll
  for (int r0 = 0; r0 < NV; r0 += R) {
    const int nr = NV - r0 < R ? NV - r0 : R;
#pragma unroll
    for (int v = 0; v < R; ++v)
      if (v < nr) buf[(g * R + v) * 64 + lane] = x[r0 + v];
    __syncthreads();
    for (int v = g; v < nr; v += G) {
      double s = buf[v * 64 + lane];
      if (MINLAST && r0 + v == NV - 1) {  // wave-uniform branch
        for (int j = 1; j < G; ++j) {
          const double y = buf[(j * R + v) * 64 + lane];
          s = y < s ? y : s;
        }
      } else {
        for (int j = 1; j < G; ++j) s += buf[(j * R + v) * 64 + lane];
      }
      tot[v * 64 + lane] = s;
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < R; ++v)
      if (v < nr) x[r0 + v] = tot[v * 64 + lane];
  }
}

// Unrolling of the transport loop over a wave's angles: full (constant slot
// indices for the register arrays; FP32 measured 6 % faster than rolled).
#ifndef RT_UNROLL_F64
#define RT_UNROLL_F64 NS
#endif
#ifndef RT_UNROLL_F32
#define RT_UNROLL_F32 NS
#endif
// The new intensities and the per-cell outputs are written once and not read
// again by the step: with RT_STREAM_STORES they bypass the caches as
// non-temporal stores, leaving L2 to the stencil reuse and the spill.
#ifndef RT_STREAM_STORES
#define RT_STREAM_STORES 1
#endif
template <typename T>
__device__ __forceinline__ void stream_store(T *p, T v) {
  if constexpr (RT_STREAM_STORES)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

// The temperature and scattering solve on every wave (1) or on wave 0 with
// the solution passed through LDS (0): FP64 on wave 0 measured 1 % faster,
// FP32 the same either way.
#ifndef RT_SOLVE_ALL_F64
#define RT_SOLVE_ALL_F64 0
#endif
#ifndef RT_SOLVE_ALL_F32
#define RT_SOLVE_ALL_F32 1
#endif
// Per-cell fields loaded before the last axis of the transport (1) or after
// the transport (0: fewer registers live in the transport, which lets FP64
// run three waves per SIMD).
#ifndef RT_CELL_EARLY_F64
#define RT_CELL_EARLY_F64 0
#endif
#ifndef RT_CELL_EARLY_F32
#define RT_CELL_EARLY_F32 0
#endif
// Transport loads of padding slots and slots with mu_d = 0: skipped by a
// wave-uniform branch (0), or issued from the last plane and weighted by the
// zero factor (1).  Plane reads by buffer loads (1) or global loads (0).
#ifndef RT_UNCOND_LOADS
#define RT_UNCOND_LOADS 0
#endif
// A scheduling fence at the start of every slot of the transport keeps the
// plane reads where the prefetch ring puts them (FP64 3.69 -> 3.61 ms,
// FP32 1.81 -> 1.79 ms with eight slots ahead, and fewer registers).
#ifndef RT_SLOT_FENCE
#define RT_SLOT_FENCE 1
#endif
#ifndef RT_BUFFER_LOADS
#define RT_BUFFER_LOADS 1
#endif
// The cell's intensities held in registers over the transport (1) or read
// again per slot (0, from L1: the center cell shares its lines with the
// neighbour reads).  FP64 reads them again, which with the per-cell fields
// after the transport fits three waves per SIMD in 168 VGPRs (3.17 -> 2.76
// ms on the 128^3 S8 box); FP32 keeps them (4 % slower reading again at
// four waves).
#ifndef RT_IC_REG_F64
#define RT_IC_REG_F64 0
#endif
#ifndef RT_IC_REG_F32
#define RT_IC_REG_F32 1
#endif
// Slots whose plane reads are in flight ahead of the transport arithmetic:
// FP32 eight (six against three: 1.88 -> 1.82 ms on the 128^3 S8 box,
// eight with the slot fence a further 1 %); FP64 five, the most that three
// waves per SIMD hold without spilling (2.80 ms at three and four, 2.76 at
// five).
#ifndef RT_PREFETCH_F64
#define RT_PREFETCH_F64 5
#endif
// (FP64 with three or four groups per wave: two, as its registers allow)
#ifndef RT_PREFETCH_F64_WIDE
#define RT_PREFETCH_F64_WIDE 2
#endif
#ifndef RT_PREFETCH_F32
#define RT_PREFETCH_F32 8
#endif

// Entry i of an angle table in the arithmetic type: the FP32 copy (equal to
// the conversion of the FP64 entry) saves a conversion per use.
template <typename A>
__device__ __forceinline__ A tab(const double *d, const float *f, int i) {
  if constexpr (sizeof(A) == 4)
    return f[i];
  else
    return d[i];
}

// A pointer into the constant address space: the angle records are read-only
// for the whole step, and reads through such a pointer at a wave-uniform
// address become scalar loads even after the step's global writes and
// atomics (through a generic pointer the compiler makes vector loads of
// them there).  128^3 S8: FP64 3.56 -> 3.18 ms, FP32 1.79 -> 1.58 ms.
#ifndef RT_CONST_RECORDS
#define RT_CONST_RECORDS 1
#endif
#if RT_CONST_RECORDS
template <typename T>
using cptr = const __attribute__((address_space(4))) T *;
#else
template <typename T>
using cptr = const T *;
#endif

// The record of angle m (StepArgs::arec) in the arithmetic type.
template <typename A>
__device__ __forceinline__ cptr<A> angle_rec(const StepArgs &p, int m) {
  if constexpr (sizeof(A) == 4)
    return (cptr<A>)(p.arecf + (size_t)m * kRec);
  else
    return (cptr<A>)(p.arec + (size_t)m * kRec);
}

// The axis data of a tile in LDS during the transport (the same bytes hold
// the reductions afterwards): per axis 8 words of cell indices and ghost
// kinds and 20 values of the arithmetic type, each a row of 64 lanes.
constexpr int kAxisWords = 8, kAxisVals = 20;
__host__ __device__ constexpr size_t axis_lds_bytes(int abytes) {
  return (size_t)3 * 64 * (kAxisWords * 4 + kAxisVals * (size_t)abytes);
}

// LDS of one step body, for G waves and abytes-byte arithmetic (dynamic
// shared memory of the launch): the cross-wave reduction rows
// (G*kChunk*64 doubles), the reduced values (kChunk*64) and the solution
// passed on by wave 0 (6*64), or the axis data of the transport if larger.
__host__ __device__ constexpr size_t step3_lds_bytes(int G, int abytes) {
  const size_t red = sizeof(double) * ((size_t)G * kChunk * 64 + kChunk * 64 + 6 * 64);
  const size_t ax = axis_lds_bytes(abytes);
  return red > ax ? red : ax;
}

// Axis d's data of the tile: stored by the wave that built it, read by every
// wave (lane by lane, so the 64 lanes hit 64 consecutive words).
template <typename A>
__device__ __forceinline__ void axis_put(double *lds, int d, const AxisData<A> &s, int lane) {
  char *base = reinterpret_cast<char *>(lds) + (size_t)d * 64 * (kAxisWords * 4 + kAxisVals * sizeof(A));
  int *w = reinterpret_cast<int *>(base);
  A *v = reinterpret_cast<A *>(base + 64 * kAxisWords * 4);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    w[j * 64 + lane] = (int)s.idx[j];
    w[(4 + j) * 64 + lane] = s.kind[j];
  }
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int t = 0; t < 3; ++t) v[(j * 3 + t) * 64 + lane] = s.dW[j][t];
  const A co[8] = {s.caL, s.cbL, s.caR, s.cbR, s.lL, s.rR, s.fL, s.fR};
#pragma unroll
  for (int j = 0; j < 8; ++j) v[(12 + j) * 64 + lane] = co[j];
}
template <typename A, bool PER>
__device__ __forceinline__ void axis_get(const double *lds, int d, AxisData<A> &s, int lane) {
  const char *base =
      reinterpret_cast<const char *>(lds) + (size_t)d * 64 * (kAxisWords * 4 + kAxisVals * sizeof(A));
  const int *w = reinterpret_cast<const int *>(base);
  const A *v = reinterpret_cast<const A *>(base + 64 * kAxisWords * 4);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    s.idx[j] = (unsigned)w[j * 64 + lane];
    s.kind[j] = PER ? 0 : w[(4 + j) * 64 + lane];
  }
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int t = 0; t < 3; ++t) s.dW[j][t] = v[(j * 3 + t) * 64 + lane];
  s.caL = v[12 * 64 + lane];
  s.cbL = v[13 * 64 + lane];
  s.caR = v[14 * 64 + lane];
  s.cbR = v[15 * 64 + lane];
  s.lL = v[16 * 64 + lane];
  s.rR = v[17 * 64 + lane];
  s.fL = v[18 * 64 + lane];
  s.fR = v[19 * 64 + lane];
}

// The reduced absorption system of one cell (Section 4.3, Eq.
// absorptionmatrix): from the angle sums S[0..8] (sum W r/D, W e/D, W/D,
// the same weighted by n.u and by u^2 + (n.u)^2) the temperature equation is
// one quartic, c_v (T' - T^n) = h0 + h1q T'^4, solved by Newton's method in
// FP64 from T^n; returns T' and sets X = T'^4/(4 pi), Q (the n.u-weighted
// intensity sum of the solution), the iteration count and convergence.
template <int NV>
__device__ __forceinline__ double absorb_solve(const StepArgs &p, const double (&S)[NV], double kap,
                                               double uu, double cv, double Tn, double sa,
                                               double &X, double &Q, int &it, bool &conv) {
  const double C = p.C, P = p.P, dt = p.dt, iC = p.invC;
  const double qden = 1.0 + kap * S[8];
  const double iqden = fast_rcp(qden);
  const double q0 = S[6] * iqden, q1 = S[7] * iqden;
  const double j0 = S[0] - kap * S[2] * q0, j1 = S[1] - kap * S[2] * q1;
  const double k0 = S[3] - kap * S[5] * q0, k1 = S[4] - kap * S[5] * q1;
  const double beta = P * C * (1.0 - uu * iC * iC) * sa * dt;
  const double g8 = 8.0 * kPi * P * sa * dt;
  const double h0 = -g8 * (k0 - q0 * iC) + kFourPi * beta * j0;
  const double h1q = (-g8 * (k1 - q1 * iC) - kFourPi * beta * (1.0 - j1)) * (1.0 / kFourPi);
  double T = Tn;
  conv = false;
  for (it = 1; it <= p.maxit; ++it) {
    const double T3 = T * T * T;
    const double f = cv * (T - Tn) - h0 - h1q * T3 * T;
    const double dT = f * fast_rcp(cv - 4.0 * h1q * T3);
    T -= dT;
    if (fabs(dT) <= p.rtol * fabs(T)) {
      conv = true;
      break;
    }
  }
  X = T * T * T * T * (1.0 / kFourPi);
  Q = q0 + q1 * X;
  return T;
}

// One step for the 64 cells of tile blk (cells blk*64 + lane), G waves.
// Writes I^{n+1}, the moments and the outputs of those cells and the tile's
// partial totals into row blk of p.partials.
template <typename S, typename A, int KA, int NG, bool PER, bool FUSED, bool SO = false>
__device__ __forceinline__ void step3_tile(const StepArgs &p, int blk, int G, double *lds) {
  constexpr int NS = KA * NG;  // angle slots of a wave: slot j*KA + k
  double *sbuf = lds, *stot = lds + (size_t)G * kChunk * 64, *ssol = stot + kChunk * 64;
  const int lane = threadIdx.x & 63;
  // wave index, made provably wave-uniform so that the angle of a slot, the
  // direction cosines and the plane offsets live in scalar registers
  const int g = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int c0 = blk * 64 + lane;
  const bool act = c0 < p.ncell;
  const int c = act ? c0 : p.ncell - 1;  // idle lanes shadow the last cell
  const int NA = p.nang;
  const size_t N = (size_t)p.ncell;
  const S *Iin = static_cast<const S *>(p.I_in);
  S *Iout = static_cast<S *>(p.I_out);
  const double C = p.C, P = p.P, dt = p.dt, iC = p.invC;
  // angle of a slot (wave-uniform), m0 + slot_off(s): valid when < NA.  The
  // slot's angle record and intensity plane are offsets from the wave's
  // first (constant offsets when the wave has one group).
  const int m0 = g * KA;
  auto slot_off = [&](int s) { return (s / KA) * G * KA + (s % KA); };
  auto slot_m = [&](int s) { return m0 + slot_off(s); };
  const cptr<A> Rg = angle_rec<A>(p, m0);
  const cptr<double> Rgd = (cptr<double>)(p.arec + (size_t)m0 * kRec);
  const S *Ig = Iin + (size_t)m0 * N;
  S *Og = Iout + (size_t)m0 * N;
  auto slot_rec = [&](int s) { return Rg + (unsigned)slot_off(s) * kRec; };
  // the sign bits of a slot's direction (scalar integer tests)
  auto slot_flags = [&](int s) -> unsigned {
    return ((cptr<unsigned>)(Rg + (unsigned)slot_off(s) * kRec + rec_flags))[0];
  };
  auto slot_plane = [&](int s) { return Ig + (size_t)(unsigned)slot_off(s) * N; };

  // The cell's fields and the moments of I^n used by the velocity estimate.
  // Loaded before the transport of the last active axis (CELL_EARLY), so
  // that their latency overlaps that axis's work, or after the transport.
  constexpr bool CELL_EARLY = sizeof(A) == 8 ? RT_CELL_EARLY_F64 : RT_CELL_EARLY_F32;
  struct {
    double sa, ss, rho, Tn, v[3], E, F[3], P[3];
  } ci;
  auto cell_load = [&]() {
    ci.sa = p.sa[c];
    ci.ss = p.ss[c];
    ci.rho = p.rho[c];
    ci.Tn = p.T[c];
#pragma unroll
    for (int k = 0; k < 3; ++k) ci.v[k] = p.v[(size_t)k * N + c];
    if (p.estimate_v) {
      ci.E = p.mom_in[c];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        ci.F[k] = p.mom_in[(size_t)(1 + k) * N + c];
        ci.P[k] = p.mom_in[(size_t)(4 + k) * N + c];
      }
    } else {
      ci.E = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) ci.F[k] = ci.P[k] = 0.0;
    }
  };

  // ------------------------------------------------ phase A: transport
  // The cell's intensities of the wave's slots: held in registers (IC_REG),
  // or read again with each slot's stencil reads (they are in L1), which
  // leaves the registers to the transport.
  constexpr bool IC_REG = sizeof(A) == 8 ? RT_IC_REG_F64 : RT_IC_REG_F32;
  A Ic[IC_REG ? NS : 1], dF[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    if constexpr (IC_REG) {
      const int m = slot_m(s);
      Ic[s] = m < NA ? A(plane_ld(slot_plane(s), (unsigned)c)) : A(0);
    }
    dF[s] = A(0);
  }
  if (FUSED) {
    const int q[3] = {c % p.n[0], (c / p.n[0]) % p.n[1], c / (p.n[0] * p.n[1])};
    const A invC = A(p.invC);
    // the axis data of the tile, each axis built by one wave (wave g takes
    // axes g, g + G, ...) and shared through LDS
    {
      const A Wc[3] = {A(p.mom_in[10 * N + c]), A(p.mom_in[11 * N + c]),
                       A(p.mom_in[12 * N + c])};
      for (int d = g; d < p.ndim; d += G) {
        AxisData<A> s;
        load_axis<A, PER>(p, c, q, d, Wc, s);
        axis_put(lds, d, s, lane);
      }
    }
    __syncthreads();
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (d >= p.ndim) break;
      if (CELL_EARLY && d == p.ndim - 1) cell_load();
      AxisData<A> s;
      axis_get<A, PER>(lds, d, s, lane);
      // does any lane of the wave have a ghost cell along this axis
      const bool ghosts =
          !PER && __any(s.kind[0] | s.kind[1] | s.kind[2] | s.kind[3]) != 0;
      constexpr int UNR = sizeof(A) == 8 ? RT_UNROLL_F64 : RT_UNROLL_F32;
      // the plane reads of a slot: cells -1 and +1 and the far upwind cell
      // (-2 for mu_d > 0, else +2).  Those of the PF next slots of the axis
      // are issued before the arithmetic of the current one, so that their
      // latency overlaps it.  (Carrying the ring across the end of an axis
      // into the next one measured slower.)
      auto reads = [&](int k, S (&r)[4]) {
        if (RT_UNCOND_LOADS || slot_m(k) < NA) {
          const S *Im = slot_m(k) < NA ? slot_plane(k) : Iin + (size_t)(NA - 1) * N;
          const unsigned far = (slot_flags(k) >> d) & 1u ? s.idx[0] : s.idx[3];
          if constexpr (RT_BUFFER_LOADS) {
            r[0] = plane_buf_ld(Im, s.idx[1]);
            r[1] = plane_buf_ld(Im, s.idx[2]);
            r[2] = plane_buf_ld(Im, far);
            if constexpr (!IC_REG) r[3] = plane_buf_ld(Im, (unsigned)c);
          } else {
            r[0] = plane_ld(Im, s.idx[1]);
            r[1] = plane_ld(Im, s.idx[2]);
            r[2] = plane_ld(Im, far);
            if constexpr (!IC_REG) r[3] = plane_ld(Im, (unsigned)c);
          }
        } else {
          r[0] = r[1] = r[2] = r[3] = S(0);
        }
      };
      constexpr int PF0 = sizeof(A) == 4 ? RT_PREFETCH_F32
                          : NG <= 2     ? RT_PREFETCH_F64
                                        : RT_PREFETCH_F64_WIDE;
      constexpr int PF = PF0 < NS ? PF0 : NS;
      S rq[PF][4];
#pragma unroll
      for (int j = 0; j < PF; ++j) reads(j, rq[j]);
#pragma unroll UNR
      for (int k = 0; k < NS; ++k) {
        if constexpr (RT_SLOT_FENCE) __builtin_amdgcn_sched_barrier(0);
        S r[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) r[t] = rq[0][t];
#pragma unroll
        for (int j = 0; j + 1 < PF; ++j)
#pragma unroll
          for (int t = 0; t < 4; ++t) rq[j][t] = rq[j + 1][t];
        if (k + PF < NS) reads(k + PF, rq[PF - 1]);
        const int m = slot_m(k);
        const int mc = m < NA ? m : NA - 1;
        const cptr<A> R = slot_rec(k);  // padding slots: zero records
        const A mud = R[rec_n0 + d];
        const unsigned fl = slot_flags(k);
        if (RT_UNCOND_LOADS || (m < NA && ((fl >> (3 + d)) & 1u))) {  // mu_d != 0, uniform
          const A n0 = R[rec_n0], n1 = R[rec_n1], n2 = R[rec_n2];
          const A h2 = R[rec_h0 + d];  // 1 - nu
          // differences of IV = n.W between consecutive stencil cells
          A V[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) V[j] = n0 * s.dW[j][0] + n1 * s.dW[j][1] + n2 * s.dW[j][2];
          const A Im1 = plane_value<S, A, PER>(p, r[0], s.idx[1], s.kind[1], 0, d, mc, mud, ghosts);
          const A Ip1 = plane_value<S, A, PER>(p, r[1], s.idx[2], s.kind[2], 1, d, mc, mud, ghosts);
          const A ick = IC_REG ? Ic[IC_REG ? k : 0] : A(r[3]);
          const A D1 = (ick - Im1) - V[1] * invC;
          const A D2 = (Ip1 - ick) - V[2] * invC;
          A T;
          if ((fl >> d) & 1u) {  // mu_d > 0
            const A Im2 = plane_value<S, A, PER>(p, r[2], s.idx[0], s.kind[0], 0, d, mc, mud, ghosts);
            const A D0 = (Im1 - Im2) - V[0] * invC;
            const A qm = vl_half(D0, D1), q0 = vl_half(D1, D2);
            T = s.cbR * D2 + (s.caL + s.cbL) * D1 + h2 * (s.caR * q0 - s.caL * qm);
          } else {
            const A Ip2 = plane_value<S, A, PER>(p, r[2], s.idx[3], s.kind[3], 1, d, mc, mud, ghosts);
            const A D3 = (Ip2 - Ip1) - V[3] * invC;
            const A q0 = vl_half(D1, D2), qp = vl_half(D2, D3);
            T = (s.caR + s.cbR) * D2 + s.cbL * D1 - h2 * (s.caR * qp - s.caL * q0);
          }
          // IV faces: the upwind cell of each face by the sign of its flow
          const A qvL = vl_half(s.fL > A(0) ? V[0] : V[2], V[1]);
          const A qvR = vl_half(s.fR > A(0) ? V[1] : V[3], V[2]);
          T += s.rR * V[2] + s.lL * V[1] + (s.fR * qvR - s.fL * qvL);
          dF[k] -= mud * T;
        }
      }
    }
    __syncthreads();  // the reductions below reuse the LDS of the axis data
  } else {
    const S *dFin = static_cast<const S *>(p.dF_in);
    if (dFin) {
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        const int m = slot_m(k);
        if (m < NA) dF[k] = A(dFin[(size_t)m * N + c]);
      }
    }
  }

  if (!(FUSED && CELL_EARLY)) cell_load();
  const double sa = ci.sa, ss = ci.ss, rho = ci.rho, Tn = ci.Tn;
  const double v0 = ci.v[0], v1 = ci.v[1], v2 = ci.v[2];

  // ---------------------------------- Step 3: velocity estimate (per cell)
  double u0 = v0, u1 = v1, u2 = v2;
  if (p.estimate_v) {
    const double h = 0.5 * dt * (sa + ss);
    const double E = ci.E, F0 = ci.F[0], F1 = ci.F[1], F2 = ci.F[2];
    const double P0 = ci.P[0], P1 = ci.P[1], P2 = ci.P[2];
    const double base = rho + h * C * rho;
    const double hPC = h * P * iC;
    u0 = (rho * v0 + h * (C * rho * v0 + P * F0)) * fast_rcp(base + hPC * (E + P0));
    u1 = (rho * v1 + h * (C * rho * v1 + P * F1)) * fast_rcp(base + hPC * (E + P1));
    u2 = (rho * v2 + h * (C * rho * v2 + P * F2)) * fast_rcp(base + hPC * (E + P2));
  }
  const double uu = u0 * u0 + u1 * u1 + u2 * u2;
  const bool to5 = ss > sa;  // Step 2 routing

  // ------------------------------------------------ phase B: source sums
  const A Au0 = A(u0), Au1 = A(u1), Au2 = A(u2), Auu = A(uu);
  const A dsa = A(dt * sa), dss = A(dt * ss);
  const A D0 = A(1.0 + dt * sa * C), E0 = A(dt * sa * C), AW0 = A(1.0 + dt * C * ss);
  const A B0 = A(-dt * C * ss - dt * ss * uu * iC), dssC = A(dt * ss * iC);
  // the routing as factors: r4 = I + g4 dF, p = r4/D + g5 dF
  const A g4 = to5 ? A(0) : A(1), g5 = to5 ? A(1) : A(0);
  const double kap = dt * sa * iC;
  const double cv = rho * p.cvfac;
  auto cell_ic = [&](int k) -> A {
    return IC_REG ? Ic[IC_REG ? k : 0] : A(plane_ld(slot_plane(k), (unsigned)c));
  };

  // SO: the absorption system is first solved at u alone (its sums and, for
  // the momentum change of that solution, sum W n (I' - r4) in closed form
  // from I'_m - r4_m = (-dt sa (C - t) r4_m + e_m X - kappa Q)/D_m), which
  // gives the time-centred velocity uc = v + d4/(2 rho) (d4 as the gas sees
  // it); the step's absorption coefficients are then taken at uc, the
  // scattering ones at u.
  double ua0 = u0, ua1 = u1, ua2 = u2, uua = uu;
  int it_first = 0;
  bool conv_first = true;
  if constexpr (SO) {
    A s1a[9], hm[9];
#pragma unroll
    for (int r = 0; r < 9; ++r) s1a[r] = hm[r] = A(0);
    const A AC = A(C);
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      if (slot_m(k) >= NA) continue;
      const cptr<A> R = slot_rec(k);
      const A n0 = R[rec_n0], n1 = R[rec_n1], n2 = R[rec_n2];
      const A t = n0 * Au0 + n1 * Au1 + n2 * Au2;
      const A invD = fast_rcp(D0 - dsa * t);
      const A e = E0 + A(3) * dsa * t;
      const A gg = Auu + t * t;
      const A r4 = cell_ic(k) + g4 * dF[k];
      const A WD = R[rec_w] * invD;
      s1a[0] += WD * r4;
      s1a[1] += WD * e;
      s1a[2] += WD;
      s1a[3] += WD * t * r4;
      s1a[4] += WD * t * e;
      s1a[5] += WD * t;
      s1a[6] += WD * gg * r4;
      s1a[7] += WD * gg * e;
      s1a[8] += WD * gg;
      const A wr = -(WD * dsa * (AC - t) * r4), we = WD * e;
      const A nn[3] = {n0, n1, n2};
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        hm[q] += nn[q] * wr;
        hm[3 + q] += nn[q] * we;
        hm[6 + q] += nn[q] * WD;
      }
    }
    double S1[9], H[9];
#pragma unroll
    for (int r = 0; r < 9; ++r) {
      S1[r] = double(s1a[r]);
      H[r] = double(hm[r]);
    }
    waves_reduce<9, false, kChunk>(S1, sbuf, stot, g, G, lane);
    waves_reduce<9, false, kChunk>(H, sbuf, stot, g, G, lane);
    double X1, Q1;
    bool ok1;
    int it1;
    absorb_solve(p, S1, kap, uu, cv, Tn, sa, X1, Q1, it1, ok1);
    it_first = it1;
    conv_first = ok1;
    // the Step 4 momentum change of the first solution, as the gas sees it
    const double fm = -p.gasfac * kFourPi * P * iC, h2r = 0.5 * fast_rcp(rho);
    ua0 = v0 + fm * (H[0] + X1 * H[3] - kap * Q1 * H[6]) * h2r;
    ua1 = v1 + fm * (H[1] + X1 * H[4] - kap * Q1 * H[7]) * h2r;
    ua2 = v2 + fm * (H[2] + X1 * H[5] - kap * Q1 * H[8]) * h2r;
    uua = ua0 * ua0 + ua1 * ua1 + ua2 * ua2;
  }
  const A Ua0 = A(ua0), Ua1 = A(ua1), Ua2 = A(ua2), Auua = A(uua);

  A pk[NS];
  A sm[kNsum];
#pragma unroll
  for (int r = 0; r < kNsum; ++r) sm[r] = A(0);
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    pk[k] = A(0);
    const int m = slot_m(k);
    if (m >= NA) continue;
    const cptr<A> R = slot_rec(k);
    const A n0 = R[rec_n0], n1 = R[rec_n1], n2 = R[rec_n2];
    const A Wm = R[rec_w];
    const A t = n0 * Au0 + n1 * Au1 + n2 * Au2;  // scattering: at u
    const A ta = SO ? n0 * Ua0 + n1 * Ua1 + n2 * Ua2 : t;  // absorption
    const A D = D0 - dsa * ta, aw = AW0 - dss * t;
    const A rDa = fast_rcp(D * aw);
    const A invD = aw * rDa, invaw = D * rDa;
    const A e = E0 + A(3) * dsa * ta;
    const A gg = (SO ? Auua : Auu) + ta * ta;
    const A b = B0 + A(2) * dss * t - dssC * t * t;
    const A cm = A(-3) * dss * t;
    const A ick = cell_ic(k);
    const A r4 = ick + g4 * dF[k];
    const A pm = r4 * invD + g5 * dF[k];
    pk[k] = pm;
    const A WD = Wm * invD, Wa = Wm * invaw, Wad = Wa * invD;
    sm[0] += WD * r4;
    sm[1] += WD * e;
    sm[2] += WD;
    sm[3] += WD * ta * r4;
    sm[4] += WD * ta * e;
    sm[5] += WD * ta;
    sm[6] += WD * gg * r4;
    sm[7] += WD * gg * e;
    sm[8] += WD * gg;
    sm[9] += Wa * b * pm;
    sm[10] += Wa * pm;
    sm[11] += Wa * b;
    sm[12] += Wa * b * cm;
    sm[13] += Wa;
    sm[14] += Wa * cm;
    sm[15] += Wad * b * e;
    sm[16] += Wad * b;
    sm[17] += Wad * e;
    sm[18] += Wad;
    const A Ir = ick + dF[k];
    sm[19] += R[rec_wn0] * Ir;
    sm[20] += R[rec_wn1] * Ir;
    sm[21] += R[rec_wn2] * Ir;
  }
  double Sa[kChunk], Sb[kChunk];
#pragma unroll
  for (int r = 0; r < kChunk; ++r) {
    Sa[r] = double(sm[r]);
    Sb[r] = double(sm[kChunk + r]);
  }
  waves_reduce<kChunk, false, kChunk>(Sa, sbuf, stot, g, G, lane);
  waves_reduce<kChunk, false, kChunk>(Sb, sbuf, stot, g, G, lane);
  // Sa = sums 0..10, Sb = sums 11..21

  // --------------------------------------------- solve (FP64)
  // Every wave holds the reduced sums of its 64 cells, so every wave can
  // solve them (SOLVE_ALL, no barrier and no idle waves), or wave 0
  // solves and passes the solution on through LDS.
  double X = 0.0, kQ = 0.0, s1 = 0.0, s2 = 0.0, T = 0.0, newton_it = 0.0;
  constexpr bool SOLVE_ALL = sizeof(A) == 8 ? RT_SOLVE_ALL_F64 : RT_SOLVE_ALL_F32;
  if (SOLVE_ALL || g == 0) {
    double Q;
    int it;
    bool conv;
    T = absorb_solve(p, Sa, kap, SO ? uua : uu, cv, Tn, sa, X, Q, it, conv);
    if (SO) {
      it = it > it_first ? it : it_first;
      conv = conv && conv_first;
    }
    if (g == 0 && act && (!conv || !(T > 0.0) || !isfinite(T))) atomicOr(p.status, 1);
    const double Sbr = Sa[9] + X * Sb[4] - kap * Q * Sb[5];
    const double Sr5 = Sa[10] + X * Sb[6] - kap * Q * Sb[7];
    const double a11 = 1.0 + Sb[0], a12 = Sb[1], a21 = Sb[2], a22 = 1.0 + Sb[3];
    const double det = a11 * a22 - a12 * a21;
    const double idet = fast_rcp(det);
    kQ = kap * Q;
    s1 = (Sbr * a22 - a12 * Sr5) * idet;
    s2 = (a11 * Sr5 - a21 * Sbr) * idet;
    newton_it = double(it);
  }
  if constexpr (!SOLVE_ALL) {
    if (g == 0) {
      ssol[0 * 64 + lane] = X;
      ssol[1 * 64 + lane] = kQ;
      ssol[2 * 64 + lane] = s1;
      ssol[3 * 64 + lane] = s2;
      ssol[4 * 64 + lane] = T;
      ssol[5 * 64 + lane] = newton_it;
    }
    __syncthreads();
    X = ssol[lane];
    kQ = ssol[64 + lane];
    s1 = ssol[128 + lane];
    s2 = ssol[192 + lane];
    T = ssol[256 + lane];
    newton_it = ssol[320 + lane];
  }

  // the sums of the earlier steps of the call that this wave's outputs add
  // to, loaded here so that their latency overlaps phase C
  double accE = 0.0, accM[3] = {0.0, 0.0, 0.0};
  if (p.accumulate) {
    if (p.dEgas && 14 % G == g) accE = p.dEgas[c];
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (p.dMom && (15 + k) % G == g) accM[k] = p.dMom[(size_t)k * N + c];
  }

  // --------------------------------------- phase C: new intensities
  const A AX = A(X), AkQ = A(kQ), As1 = A(s1), As2 = A(s2);
  double mo[kChunk];
#pragma unroll
  for (int r = 0; r < 10; ++r) mo[r] = 0.0;
  mo[10] = 1.0e300;
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const int m = slot_m(k);
    if (m >= NA) continue;
    const cptr<A> R = slot_rec(k);
    const A t = R[rec_n0] * Au0 + R[rec_n1] * Au1 + R[rec_n2] * Au2;
    const A ta = SO ? R[rec_n0] * Ua0 + R[rec_n1] * Ua1 + R[rec_n2] * Ua2 : t;
    const A D = D0 - dsa * ta, aw = AW0 - dss * t;
    const A rDa = fast_rcp(D * aw);
    const A e = E0 + A(3) * dsa * ta;
    const A cm = A(-3) * dss * t;
    // I' = invaw (p - s1 - c s2) + invD invaw (e X - kappa Q)
    const S Inew = S(D * rDa * (pk[k] - As1 - cm * As2) + rDa * (e * AX - AkQ));
    if (act) stream_store(&Og[(size_t)(unsigned)slot_off(k) * N + c], Inew);
    // the quadrature of Section 3: w, w n_i and w n_i n_j from the table
    const double In = double(Inew);
#pragma unroll
    for (int r = 0; r < 10; ++r) mo[r] += Rgd[(unsigned)slot_off(k) * kRec + rec_w + r] * In;
    mo[10] = In < mo[10] ? In : mo[10];
  }
  waves_reduce<kChunk, true, kChunk>(mo, sbuf, stot, g, G, lane);
#pragma unroll
  for (int r = 0; r < 10; ++r) mo[r] *= kFourPi;

  // ------------------------------------------------ Step 7 and outputs
  // the gas changes: gasfac (C over the reduced speed, 1 without one) times
  // the momentum the radiation loses, and the true heat capacity
  const double PC = P * iC, f4 = kFourPi * PC, gf = p.gasfac;
  const double irho = fast_rcp(rho);
  const double dm0 = gf * (-PC * mo[1] + f4 * Sb[8]);
  const double dm1 = gf * (-PC * mo[2] + f4 * Sb[9]);
  const double dm2 = gf * (-PC * mo[3] + f4 * Sb[10]);
  const double mm0 = rho * v0, mm1 = rho * v1, mm2 = rho * v2;
  const double ek =
      (((mm0 + dm0) * (mm0 + dm0) + (mm1 + dm1) * (mm1 + dm1) + (mm2 + dm2) * (mm2 + dm2)) -
       (mm0 * mm0 + mm1 * mm1 + mm2 * mm2)) *
      (0.5 * irho);
  const double cvg = cv * gf;
  const double deg = cvg * (T - Tn) + ek;
  // gas feedback (rho fixed): the momentum change of the step moves the flow;
  // 3 v J of the new state, used by the next step's IV, takes the new v
  const double vn0 = p.feedback ? v0 + dm0 * irho : v0;
  const double vn1 = p.feedback ? v1 + dm1 * irho : v1;
  const double vn2 = p.feedback ? v2 + dm2 * irho : v2;
  if (act) {
    // The per-cell fields (0-9 the moments, 10-12 3vJ of the new state, 13
    // T, 14 dEgas, 15-17 dMom, 18-27 the optional output moments) are spread
    // over the waves, 64 consecutive cells each: wave g takes the fields
    // f = g mod G.  The loop is unrolled so that every field number is a
    // constant (no dynamic indexing of mo[]).  With FP32 storage the
    // wave's share is tested on a uniform bit mask; FP64 storage, short of
    // registers, measured faster with the remainder taken per field.
    unsigned fmask = 0u;
    if constexpr (sizeof(S) == 4)
      for (int f = g; f < 28; f += G) fmask |= 1u << f;
#pragma unroll
    for (int f = 0; f < 28; ++f) {
      if (sizeof(S) == 4 ? !((fmask >> f) & 1u) : f % G != g) continue;
      double val;
      double *dst;
      if (f < 10) {
        val = mo[f];
        dst = p.mom_out + (size_t)f * N;
      } else if (f < 13) {
        val = p.ivfac * (f == 10 ? vn0 : f == 11 ? vn1 : vn2) * mo[0] * (1.0 / kFourPi);
        dst = p.mom_out + (size_t)f * N;
      } else if (f == 13) {
        val = T;
        dst = p.T;
      } else if (f == 14) {
        if (!p.dEgas) continue;
        val = accE + deg;
        dst = p.dEgas;
      } else if (f < 18) {
        if (!p.dMom) continue;
        const int k = f - 15;
        val = accM[k] + (k == 0 ? dm0 : k == 1 ? dm1 : dm2);
        dst = p.dMom + (size_t)k * N;
      } else if (f == 18) {
        if (!p.oE) continue;
        val = mo[0];
        dst = p.oE;
      } else if (f < 22) {
        if (!p.oF) continue;
        val = mo[f - 18];
        dst = p.oF + (size_t)(f - 19) * N;
      } else {
        if (!p.oP) continue;
        val = mo[f - 18];
        dst = p.oP + (size_t)(f - 22) * N;
      }
      stream_store(&dst[c], val);
    }
    // gas feedback: the new velocity (every wave has read this cell's v
    // before the reductions above)
    if (p.feedback && g == G - 1) {
      p.v[c] = vn0;
      p.v[N + c] = vn1;
      p.v[2 * N + c] = vn2;
    }
  }
  if (g == 0) {
    double tot[kNtot];
    const double vol = p.vol;
    const bool on = act;
    tot[0] = on ? P * mo[0] * vol : 0.0;
    tot[1] = on ? cvg * T * vol : 0.0;
    tot[2] = on ? deg * vol : 0.0;
    tot[3] = on ? ek * vol : 0.0;
    tot[4] = on ? dm0 * vol : 0.0;
    tot[5] = on ? dm1 * vol : 0.0;
    tot[6] = on ? dm2 * vol : 0.0;
    tot[7] = on ? PC * mo[1] * vol : 0.0;
    tot[8] = on ? PC * mo[2] * vol : 0.0;
    tot[9] = on ? PC * mo[3] * vol : 0.0;
    tot[10] = on ? mo[10] : 1.0e300;
    tot[11] = on ? newton_it : 0.0;
#pragma unroll
    for (int k = 0; k < kNtot; ++k) {
      const double x = (k == 10) ? wave_min(tot[k]) : (k == 11) ? wave_max(tot[k]) : wave_sum(tot[k]);
      if (lane == 0) store_partial(p.partials, p.nparts, blk, k, x, p.accumulate);
    }
  }
}

// Waves per SIMD the register allocation of k_step3 targets.  FP64 at 3
// (168 VGPRs: the cell's intensities read again per slot and the per-cell
// fields after the transport; with 4-wave blocks three blocks share a CU)
// against 2 (256 VGPRs): 2.76 against 3.17 ms on the 128^3 S8 box; at 4
// it spills.  FP32 at 4 does not spill (at 5 it does).
#ifndef RT_STEP3_WAVES_F64
#define RT_STEP3_WAVES_F64 3
#endif
#ifndef RT_STEP3_WAVES_F32
#define RT_STEP3_WAVES_F32 4
#endif

// Order of the tiles over the blocks: 0 dispatch order, 1 XCD-contiguous,
// 2 XCD slabs of z-planes with z fastest (slab_block), 3, 4, 5 the same in
// sub-slabs of 4, 8, 2 planes.  Both take sub-slabs of 4: on the 128^3 S8
// box FP64 (three 40 KB tiles of intensities per CU in flight) 2.77 -> 2.72
// ms with the fetched bytes 9.7 -> 5.1 GB, FP32 the same time with 4.0 ->
// 2.3 GB fetched.
#ifndef RT_BLOCK_ORDER_F64
#define RT_BLOCK_ORDER_F64 3
#endif
#ifndef RT_BLOCK_ORDER_F32
#define RT_BLOCK_ORDER_F32 3
#endif

template <typename S, typename A, int KA, int NG, bool PER, bool FUSED, bool SO = false>
__global__ __launch_bounds__(64 * kMaxWaves, sizeof(S) == 8 ? RT_STEP3_WAVES_F64
                                                            : RT_STEP3_WAVES_F32) void
k_step3(StepArgs p) {
  extern __shared__ double lds_[];
  constexpr int ORD = sizeof(S) == 8 ? RT_BLOCK_ORDER_F64 : RT_BLOCK_ORDER_F32;
  const int b = (int)blockIdx.x, nb = (int)gridDim.x;
  const int blk = ORD >= 2   ? slab_block(b, nb, p.n, ORD == 2 ? 0 : ORD == 3 ? 4 : ORD == 4 ? 8 : 2)
                  : ORD == 1 ? xcd_block(b, nb)
                             : b;
  step3_tile<S, A, KA, NG, PER, FUSED, SO>(p, blk, blockDim.x >> 6, lds_);
}

// A whole solve per workgroup: job blockIdx.x advances its grid through
// nsteps fused steps, tile by tile (64 cells per tile, the waves of the
// context's launch shape, the same step body as k_step3, hence the same
// per-cell results and partial totals), and reduces the partial totals
// after the last step like k_totals.  Between steps the workgroup fences its global writes (I,
// moments, T, partials) before any wave reads them.
template <typename S, typename A, int KA, int NG, bool PER>
__global__ __launch_bounds__(64 * kMaxWaves) void k_step3_packed(
    const PackedJob *__restrict__ jobs) {
  extern __shared__ double lds_[];
  __shared__ double red[kNtot * kVWaves];
  const PackedJob &J = jobs[blockIdx.x];
  StepArgs p = J.a;
  const int ntiles = p.nparts;
  void *Ib[2] = {const_cast<void *>(p.I_in), p.I_out};
  double *Mb[2] = {const_cast<double *>(p.mom_in), p.mom_out};
  double *oE = p.oE, *oF = p.oF, *oP = p.oP;
  for (int s = 0; s < J.nsteps; ++s) {
    const bool last = s == J.nsteps - 1;
    p.I_in = Ib[s & 1];
    p.I_out = Ib[(s + 1) & 1];
    p.mom_in = Mb[s & 1];
    p.mom_out = Mb[(s + 1) & 1];
    p.accumulate = s > 0 ? 1 : 0;
    p.oE = last ? oE : nullptr;
    p.oF = last ? oF : nullptr;
    p.oP = last ? oP : nullptr;
    for (int t = 0; t < ntiles; ++t) {
      // the tile body's first LDS writes (the axis data) may overlap the
      // reduced values the previous tile's waves are still reading
      if (t > 0) __syncthreads();
      step3_tile<S, A, KA, NG, PER, true>(p, t, blockDim.x >> 6, lds_);
    }
    __threadfence();
    __syncthreads();
  }
  if (J.totals) totals_reduce(p.partials, ntiles, J.totals, red);
}

}  // namespace rtk
