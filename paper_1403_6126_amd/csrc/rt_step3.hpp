// Fused step kernel with the waves of a block sharing cells (angle-major
// layout I[m][c]).
//
// A block holds 64 consecutive cells (one per lane) and G <= 8 waves; the
// angles are cut into groups of KA, and wave g owns the groups g, g + G, ...
// (NG of them at most, so up to NG*G*KA angles).  Within a wave the angle is
// uniform, so the direction cosines, weights and the upwind
// direction of every axis are scalars, and every intensity load reads 64
// consecutive cells of one angle plane.  Per step:
//   phase A  transport increment of the wave's angles (Section 4.2), one
//            active axis at a time, from a per-call interface table (alpha,
//            flow speed, IV Courant factor) and 3 v J carried with the
//            moments;
//   phase B  the absorption right-hand side r4 and the wave's partial sums of
//            the per-cell sums of the reduced absorption and scattering
//            systems; the per-angle values stay in registers;
//   reduce   the partial sums across the waves (LDS, fixed order);
//   solve    wave 0: FP64 Newton on the quartic in T' and the 2 x 2
//            scattering system; the solution goes to the other waves via LDS;
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

// up1 + (h2/2) * vanLeer(up1 - up2, dn1 - up1), vanLeer(a, b) = 2ab/(a + b)
// when ab > 0, else 0: the upwind interface value of the monotonic
// piecewise-linear reconstruction at Courant number nu, h2 = 1 - nu.  The
// factor 2 of the limiter and the 1/2 of the Courant factor cancel exactly
// (scaling by 2 is exact), which saves an instruction per face.
template <typename A>
__device__ __forceinline__ A vl_face(A up2, A up1, A dn1, A h2) {
  const A a = up1 - up2, b = dn1 - up1;
  const A ab = a * b;
  const A q = ab * limiter_rcp(a + b);
  return up1 + h2 * (ab > A(0) ? q : A(0));
}

// Stencil of one cell along one axis.
template <typename A>
struct Stencil {
  int idx[4];   // cells at offsets -2, -1, +1, +2 (wrapped, or the edge cell)
  int kind[4];  // 0 read the cell, 1 fixed table, 2 vacuum
  A wv[4][3];   // 3 v J at those cells
  A aL, aR, hL, hR;  // hL, hR: 1 - nu of the IV faces (twice the table's)
  A bL, bR;          // (1 - alpha)/2: the weight of the sum of the two centre values
  double uL, uR;
};

template <typename A, bool PER>
__device__ __forceinline__ void load_stencil(const StepArgs &p, int c, const int q[3], int d,
                                             Stencil<A> &s) {
  const int n = p.n[d];
  const size_t N = (size_t)p.ncell;
  const int offs[4] = {-2, -1, 1, 2};
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
    s.idx[j] = cj;
    s.kind[j] = kind;
#pragma unroll
    for (int t = 0; t < 3; ++t) s.wv[j][t] = A(p.mom_in[(size_t)(10 + t) * N + cj]);
  }
  s.aL = A(p.faces[(size_t)(d * 3 + 0) * N + c]);
  s.hL = A(p.faces[(size_t)(d * 3 + 1) * N + c]);
  s.hL += s.hL;
  s.uL = p.faces[(size_t)(d * 3 + 2) * N + c];
  if (PER || q[d] + 1 < n || p.bc[d][1] == kPeriodic) {
    const int cr = s.idx[2];
    s.aR = A(p.faces[(size_t)(d * 3 + 0) * N + cr]);
    s.hR = A(p.faces[(size_t)(d * 3 + 1) * N + cr]);
    s.hR += s.hR;
    s.uR = p.faces[(size_t)(d * 3 + 2) * N + cr];
  } else {
    // high non-periodic boundary: the ghost copies this cell's fields
    const double u = p.v[(size_t)d * N + c];
    s.aR = A(alpha_of(p.sa[c] + p.ss[c], p.dl10[d]));
    s.hR = A(0.5 * (1.0 - fabs(u) * p.dt_dx[d]));
    s.hR += s.hR;
    s.uR = u;
  }
  s.bL = A(0.5) * (A(1) - s.aL);
  s.bR = A(0.5) * (A(1) - s.aR);
}

// Intensity at a stencil cell from the value raw read at its (clamped) cell
// idx of the angle plane, with the ghost kinds.
template <typename S, typename A, bool PER>
__device__ __forceinline__ A plane_value(const StepArgs &p, S raw, int idx, int kind, int side,
                                         int d, int m, A mud) {
  if (PER || kind == 0) return A(raw);
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
      const bool mn = MINLAST && r0 + v == NV - 1;
      for (int j = 1; j < G; ++j) {
        const double y = buf[(j * R + v) * 64 + lane];
        s = mn ? fmin(s, y) : s + y;
      }
      tot[v * 64 + lane] = s;
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < R; ++v)
      if (v < nr) x[r0 + v] = tot[v * 64 + lane];
  }
}

// Unrolling of the transport loop over a wave's angles: full for FP64 (all
// loads in flight at once), none for FP32 (registers).
#ifndef RT_UNROLL_F64
#define RT_UNROLL_F64 NS
#endif
#ifndef RT_UNROLL_F32
#define RT_UNROLL_F32 1
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

// Slots whose plane reads are in flight ahead of the transport arithmetic
// (FP64 storage: one, as registers allow).
#ifndef RT_PREFETCH_F64
#define RT_PREFETCH_F64 1
#endif
#ifndef RT_PREFETCH_F32
#define RT_PREFETCH_F32 3
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

// Shared memory of one step body.
// Values per reduction round: all 11 at once (the registers, not the LDS,
// bound the blocks per CU of both storage types).
template <typename S>
struct Step3Smem {
  static constexpr int R = kChunk;
  double buf[kMaxWaves * R * 64];
  double tot[R * 64];
  double sol[6 * 64];
};

// One step for the 64 cells of tile blk (cells blk*64 + lane), G waves.
// Writes I^{n+1}, the moments and the outputs of those cells and the tile's
// partial totals into row blk of p.partials.
template <typename S, typename A, int KA, int NG, bool PER, bool FUSED>
__device__ __forceinline__ void step3_tile(const StepArgs &p, int blk, int G, Step3Smem<S> &sm_) {
  constexpr int NS = KA * NG;  // angle slots of a wave: slot j*KA + k
  double *sbuf = sm_.buf, *stot = sm_.tot, *ssol = sm_.sol;
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
  const double C = p.C, P = p.P, dt = p.dt;
  // angle of a slot (wave-uniform); valid when < NA, table reads clamped
  auto slot_m = [&](int s) { return (g + (s / KA) * G) * KA + (s % KA); };

  // ------------------------------------------------ phase A: transport
  A Ic[NS], dF[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int m = slot_m(s);
    Ic[s] = m < NA ? A(Iin[(size_t)m * N + c]) : A(0);
    dF[s] = A(0);
  }
  if (FUSED) {
    const int q[3] = {c % p.n[0], (c / p.n[0]) % p.n[1], c / (p.n[0] * p.n[1])};
    const A wc0 = A(p.mom_in[10 * N + c]), wc1 = A(p.mom_in[11 * N + c]),
            wc2 = A(p.mom_in[12 * N + c]);
    const A AC = A(C), invC = A(p.invC);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (d >= p.ndim) break;
      Stencil<A> s;
      load_stencil<A, PER>(p, c, q, d, s);
      const A dtdx = A(p.dt_dx[d]);
      const bool posR = s.uR > 0.0, posL = s.uL > 0.0;
      const bool zeroR = s.uR == 0.0, zeroL = s.uL == 0.0;
      constexpr int UNR = sizeof(A) == 8 ? RT_UNROLL_F64 : RT_UNROLL_F32;
      // the plane reads of a slot: cells -1 and +1 and the far upwind cell
      // (-2 for mu_d > 0, else +2).  Those of the PF next slots are issued
      // before the arithmetic of the current one, so that their latency
      // overlaps it.
      auto reads = [&](int k, S (&r)[3]) {
        const int m = slot_m(k);
        const int mc = m < NA ? m : NA - 1;
        const S *Im = Iin + (size_t)mc * N;
        r[0] = Im[s.idx[1]];
        r[1] = Im[s.idx[2]];
        r[2] = Im[tab<A>(p.mu, p.muf, d * NA + mc) > A(0) ? s.idx[0] : s.idx[3]];
      };
      constexpr int PF = sizeof(A) == 8 ? RT_PREFETCH_F64 : RT_PREFETCH_F32;
      S q[PF][3];
#pragma unroll
      for (int j = 0; j < PF; ++j)
        if (j < NS) reads(j, q[j]);
#pragma unroll UNR
      for (int k = 0; k < NS; ++k) {
          S r[3];
#pragma unroll
          for (int t = 0; t < 3; ++t) r[t] = q[0][t];
#pragma unroll
          for (int j = 0; j + 1 < PF; ++j)
#pragma unroll
            for (int t = 0; t < 3; ++t) q[j][t] = q[j + 1][t];
          if (k + PF < NS) reads(k + PF, q[PF - 1]);
          const int m = slot_m(k);
          const int mc = m < NA ? m : NA - 1;
          const A n0 = tab<A>(p.mu, p.muf, mc), n1 = tab<A>(p.mu, p.muf, NA + mc),
                  n2 = tab<A>(p.mu, p.muf, 2 * NA + mc);
          const A mud = d == 0 ? n0 : d == 1 ? n1 : n2;
          if (m < NA && mud != A(0)) {  // uniform over the wave
          A IV[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) IV[j] = n0 * s.wv[j][0] + n1 * s.wv[j][1] + n2 * s.wv[j][2];
          const A IVc = n0 * wc0 + n1 * wc1 + n2 * wc2;
          const A Itc = Ic[k] - IVc * invC;
          const A Im1 = plane_value<S, A, PER>(p, r[0], s.idx[1], s.kind[1], 0, d, m, mud);
          const A Ip1 = plane_value<S, A, PER>(p, r[1], s.idx[2], s.kind[2], 1, d, m, mud);
          const A Itm1 = Im1 - IV[1] * invC, Itp1 = Ip1 - IV[2] * invC;
          const A h = A(1) - AC * fabs(mud) * dtdx;  // 1 - nu
          A upR, upL;
          if (mud > A(0)) {
            const A Im2 = plane_value<S, A, PER>(p, r[2], s.idx[0], s.kind[0], 0, d, m, mud);
            const A Itm2 = Im2 - IV[0] * invC;
            upR = vl_face(Itm1, Itc, Itp1, h);
            upL = vl_face(Itm2, Itm1, Itc, h);
          } else {
            const A Ip2 = plane_value<S, A, PER>(p, r[2], s.idx[3], s.kind[3], 1, d, m, mud);
            const A Itp2 = Ip2 - IV[3] * invC;
            upR = vl_face(Itp2, Itp1, Itc, h);
            upL = vl_face(Itp1, Itc, Itm1, h);
          }
          // alpha I~*_up + (1 - alpha) I~_c of the two faces
          const A xR = s.aR * upR + s.bR * (Itc + Itp1);
          const A xL = s.aL * upL + s.bL * (Itm1 + Itc);
          A ivR, ivL;
          {
            const A u2 = posR ? IV[1] : IV[3], u1 = posR ? IVc : IV[2], d1 = posR ? IV[2] : IVc;
            const A f = vl_face(u2, u1, d1, s.hR);
            ivR = zeroR ? A(0.5) * (IVc + IV[2]) : f;
          }
          {
            const A u2 = posL ? IV[0] : IV[2], u1 = posL ? IV[1] : IVc, d1 = posL ? IVc : IV[1];
            const A f = vl_face(u2, u1, d1, s.hL);
            ivL = zeroL ? A(0.5) * (IV[1] + IVc) : f;
          }
          // the fluxes C mu x + mu IV* with mu dt/dx taken out of the difference
          dF[k] -= (dtdx * mud) * ((AC * xR + ivR) - (AC * xL + ivL));
        }
      }
    }
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

  // the cell's fields, first needed here (loaded after the transport so that
  // they take no registers there)
  const double sa = p.sa[c], ss = p.ss[c], rho = p.rho[c], Tn = p.T[c];
  const double v0 = p.v[c], v1 = p.v[N + c], v2 = p.v[2 * N + c];

  // ---------------------------------- Step 3: velocity estimate (per cell)
  double u0 = v0, u1 = v1, u2 = v2;
  if (p.estimate_v) {
    const double h = 0.5 * dt * (sa + ss);
    const double E = p.mom_in[c];
    const double F0 = p.mom_in[N + c], F1 = p.mom_in[2 * N + c], F2 = p.mom_in[3 * N + c];
    const double P0 = p.mom_in[4 * N + c], P1 = p.mom_in[5 * N + c], P2 = p.mom_in[6 * N + c];
    const double base = rho + h * C * rho;
    u0 = (rho * v0 + h * (C * rho * v0 + P * F0)) / (base + h * P * (E + P0) / C);
    u1 = (rho * v1 + h * (C * rho * v1 + P * F1)) / (base + h * P * (E + P1) / C);
    u2 = (rho * v2 + h * (C * rho * v2 + P * F2)) / (base + h * P * (E + P2) / C);
  }
  const double uu = u0 * u0 + u1 * u1 + u2 * u2;
  const bool to5 = ss > sa;  // Step 2 routing

  // ------------------------------------------------ phase B: source sums
  const A Au0 = A(u0), Au1 = A(u1), Au2 = A(u2), Auu = A(uu);
  const A dsa = A(dt * sa), dss = A(dt * ss);
  const A D0 = A(1.0 + dt * sa * C), E0 = A(dt * sa * C), AW0 = A(1.0 + dt * C * ss);
  const A B0 = A(-dt * C * ss - dt * ss * uu / C), dssC = A(dt * ss / C);
  A pk[NS];
  A sm[kNsum];
#pragma unroll
  for (int r = 0; r < kNsum; ++r) sm[r] = A(0);
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    pk[k] = A(0);
    const int m = slot_m(k);
    if (m >= NA) continue;
    const A n0 = tab<A>(p.mu, p.muf, m), n1 = tab<A>(p.mu, p.muf, NA + m),
            n2 = tab<A>(p.mu, p.muf, 2 * NA + m);
    const A Wm = tab<A>(p.w, p.wf, m);
    const A t = n0 * Au0 + n1 * Au1 + n2 * Au2;
    const A D = D0 - dsa * t, aw = AW0 - dss * t;
    const A rDa = fast_rcp(D * aw);
    const A invD = aw * rDa, invaw = D * rDa;
    const A e = E0 + A(3) * dsa * t;
    const A gg = Auu + t * t;
    const A b = B0 + A(2) * dss * t - dssC * t * t;
    const A cm = A(-3) * dss * t;
    const A r4 = to5 ? Ic[k] : Ic[k] + dF[k];
    const A pm = r4 * invD + (to5 ? dF[k] : A(0));
    pk[k] = pm;
    const A WD = Wm * invD, Wa = Wm * invaw, Wad = Wa * invD;
    sm[0] += WD * r4;
    sm[1] += WD * e;
    sm[2] += WD;
    sm[3] += WD * t * r4;
    sm[4] += WD * t * e;
    sm[5] += WD * t;
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
    const A WI = Wm * (Ic[k] + dF[k]);
    sm[19] += n0 * WI;
    sm[20] += n1 * WI;
    sm[21] += n2 * WI;
  }
  double Sa[kChunk], Sb[kChunk];
#pragma unroll
  for (int r = 0; r < kChunk; ++r) {
    Sa[r] = double(sm[r]);
    Sb[r] = double(sm[kChunk + r]);
  }
  waves_reduce<kChunk, false, Step3Smem<S>::R>(Sa, sbuf, stot, g, G, lane);
  waves_reduce<kChunk, false, Step3Smem<S>::R>(Sb, sbuf, stot, g, G, lane);
  // Sa = sums 0..10, Sb = sums 11..21

  // --------------------------------------------- solve (FP64, wave 0)
  const double kap = dt * sa / C;
  const double cv = rho * p.cvfac;
  if (g == 0) {
    const double qden = 1.0 + kap * Sa[8];
    const double q0 = Sa[6] / qden, q1 = Sa[7] / qden;
    const double j0 = Sa[0] - kap * Sa[2] * q0, j1 = Sa[1] - kap * Sa[2] * q1;
    const double k0 = Sa[3] - kap * Sa[5] * q0, k1 = Sa[4] - kap * Sa[5] * q1;
    const double beta = P * C * (1.0 - uu / (C * C)) * sa * dt;
    const double g8 = 8.0 * kPi * P * sa * dt;
    const double h0 = -g8 * (k0 - q0 / C) + kFourPi * beta * j0;
    const double h1q = (-g8 * (k1 - q1 / C) - kFourPi * beta * (1.0 - j1)) * (1.0 / kFourPi);
    double T = Tn;
    int it;
    bool conv = false;
    for (it = 1; it <= p.maxit; ++it) {
      const double T3 = T * T * T;
      const double f = cv * (T - Tn) - h0 - h1q * T3 * T;
      const double dT = f / (cv - 4.0 * h1q * T3);
      T -= dT;
      if (fabs(dT) <= p.rtol * fabs(T)) {
        conv = true;
        break;
      }
    }
    if (act && (!conv || !(T > 0.0) || !isfinite(T))) atomicOr(p.status, 1);
    const double X = T * T * T * T * (1.0 / kFourPi);
    const double Q = q0 + q1 * X;
    const double Sbr = Sa[9] + X * Sb[4] - kap * Q * Sb[5];
    const double Sr5 = Sa[10] + X * Sb[6] - kap * Q * Sb[7];
    const double a11 = 1.0 + Sb[0], a12 = Sb[1], a21 = Sb[2], a22 = 1.0 + Sb[3];
    const double det = a11 * a22 - a12 * a21;
    ssol[0 * 64 + lane] = X;
    ssol[1 * 64 + lane] = kap * Q;
    ssol[2 * 64 + lane] = (Sbr * a22 - a12 * Sr5) / det;
    ssol[3 * 64 + lane] = (a11 * Sr5 - a21 * Sbr) / det;
    ssol[4 * 64 + lane] = T;
    ssol[5 * 64 + lane] = double(it);
  }
  __syncthreads();
  const double X = ssol[lane], kQ = ssol[64 + lane], s1 = ssol[128 + lane],
               s2 = ssol[192 + lane], T = ssol[256 + lane];
  const double newton_it = ssol[320 + lane];

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
    const double d0 = p.mu[m], d1 = p.mu[NA + m], d2 = p.mu[2 * NA + m];
    const A t = tab<A>(p.mu, p.muf, m) * Au0 + tab<A>(p.mu, p.muf, NA + m) * Au1 +
                tab<A>(p.mu, p.muf, 2 * NA + m) * Au2;
    const A D = D0 - dsa * t, aw = AW0 - dss * t;
    const A rDa = fast_rcp(D * aw);
    const A e = E0 + A(3) * dsa * t;
    const A cm = A(-3) * dss * t;
    // I' = invaw (p - s1 - c s2) + invD invaw (e X - kappa Q)
    const S Inew = S(D * rDa * (pk[k] - As1 - cm * As2) + rDa * (e * AX - AkQ));
    if (act) stream_store(&Iout[(size_t)m * N + c], Inew);
    const double Iw = double(Inew) * p.w[m];
    mo[0] += Iw;
    mo[1] += d0 * Iw;
    mo[2] += d1 * Iw;
    mo[3] += d2 * Iw;
    mo[4] += d0 * d0 * Iw;
    mo[5] += d1 * d1 * Iw;
    mo[6] += d2 * d2 * Iw;
    mo[7] += d0 * d1 * Iw;
    mo[8] += d0 * d2 * Iw;
    mo[9] += d1 * d2 * Iw;
    mo[10] = fmin(mo[10], double(Inew));
  }
  waves_reduce<kChunk, true, Step3Smem<S>::R>(mo, sbuf, stot, g, G, lane);
#pragma unroll
  for (int r = 0; r < 10; ++r) mo[r] *= kFourPi;

  // ------------------------------------------------ Step 7 and outputs
  // the gas changes: gasfac (C over the reduced speed, 1 without one) times
  // the momentum the radiation loses, and the true heat capacity
  const double f4 = kFourPi * P / C, gf = p.gasfac;
  const double dm0 = gf * (-(P / C) * mo[1] + f4 * Sb[8]);
  const double dm1 = gf * (-(P / C) * mo[2] + f4 * Sb[9]);
  const double dm2 = gf * (-(P / C) * mo[3] + f4 * Sb[10]);
  const double mm0 = rho * v0, mm1 = rho * v1, mm2 = rho * v2;
  const double ek =
      (((mm0 + dm0) * (mm0 + dm0) + (mm1 + dm1) * (mm1 + dm1) + (mm2 + dm2) * (mm2 + dm2)) -
       (mm0 * mm0 + mm1 * mm1 + mm2 * mm2)) /
      (2.0 * rho);
  const double cvg = cv * gf;
  const double deg = cvg * (T - Tn) + ek;
  // gas feedback (rho fixed): the momentum change of the step moves the flow;
  // 3 v J of the new state, used by the next step's IV, takes the new v
  const double vn0 = p.feedback ? v0 + dm0 / rho : v0;
  const double vn1 = p.feedback ? v1 + dm1 / rho : v1;
  const double vn2 = p.feedback ? v2 + dm2 / rho : v2;
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
        val = (p.accumulate ? p.dEgas[c] : 0.0) + deg;
        dst = p.dEgas;
      } else if (f < 18) {
        if (!p.dMom) continue;
        const int k = f - 15;
        val = (p.accumulate ? p.dMom[(size_t)k * N + c] : 0.0) + (k == 0 ? dm0 : k == 1 ? dm1 : dm2);
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
    tot[7] = on ? P / C * mo[1] * vol : 0.0;
    tot[8] = on ? P / C * mo[2] * vol : 0.0;
    tot[9] = on ? P / C * mo[3] * vol : 0.0;
    tot[10] = on ? mo[10] : 1.0e300;
    tot[11] = on ? newton_it : 0.0;
#pragma unroll
    for (int k = 0; k < kNtot; ++k) {
      const double x = (k == 10) ? wave_min(tot[k]) : (k == 11) ? wave_max(tot[k]) : wave_sum(tot[k]);
      if (lane == 0) store_partial(p.partials, p.nparts, blk, k, x, p.accumulate);
    }
  }
}

// Waves per SIMD the register allocation of k_step3 targets (8-wave blocks:
// 2 = one block per CU, 4 = two, 6 = three).  Measured on the 128^3 S8 box:
// FP64 at 4 (128 VGPRs, a small spill) runs 5.0 ms against 6.0 ms at 2;
// FP32 at 6 (80 VGPRs) spills enough to lose to 4.
#ifndef RT_STEP3_WAVES_F64
#define RT_STEP3_WAVES_F64 4
#endif
#ifndef RT_STEP3_WAVES_F32
#define RT_STEP3_WAVES_F32 4
#endif

template <typename S, typename A, int KA, int NG, bool PER, bool FUSED>
__global__ __launch_bounds__(64 * kMaxWaves, sizeof(S) == 8 ? RT_STEP3_WAVES_F64
                                                            : RT_STEP3_WAVES_F32) void
k_step3(StepArgs p) {
  __shared__ Step3Smem<S> sm_;
  // FP32 storage gains from XCD-contiguous work; the FP64 kernel, whose
  // traffic is mostly its own spill, measured 6 % faster in dispatch order.
  const int blk = sizeof(S) == 4 ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  step3_tile<S, A, KA, NG, PER, FUSED>(p, blk, blockDim.x >> 6, sm_);
}

// A whole solve per workgroup: job blockIdx.x advances its grid through
// nsteps fused steps, tile by tile (64 cells per tile, kMaxWaves waves, the
// same step body as k_step3, hence the same per-cell results and partial
// totals), and reduces the partial totals after the last step like
// k_totals.  Between steps the workgroup fences its global writes (I,
// moments, T, partials) before any wave reads them.
template <typename S, typename A, int KA, int NG, bool PER>
__global__ __launch_bounds__(64 * kMaxWaves) void k_step3_packed(
    const PackedJob *__restrict__ jobs) {
  __shared__ Step3Smem<S> sm_;
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
    for (int t = 0; t < ntiles; ++t)
      step3_tile<S, A, KA, NG, PER, true>(p, t, kMaxWaves, sm_);
    __threadfence();
    __syncthreads();
  }
  if (J.totals) totals_reduce(p.partials, ntiles, J.totals, red);
}

}  // namespace rtk
