// Fused step kernels with the angles of a cell spread over a group of lanes.
//
// Layout: I[c][m] (cell-major, the nang angles of a cell contiguous).  A
// 256-lane block holds CPB = 256/SLOTS cells; the SLOTS lanes of a cell take
// the angles m = slot, slot + SLOTS, ... (at most KMAX per lane), so a load
// instruction reads SLOTS consecutive angles of each of the cells of a wave.
//
// Per step and cell (Section 4.1, Steps 2-5 and 7):
//   phase A  transport increment dF_m, one active axis at a time: the van
//            Leer interface values of I~ = I - IV/C (speed alpha C) and of
//            IV = 3 n.v J (flow speed), both faces of the cell;
//   phase B  absorption right-hand side r4_m and the partial sums over the
//            lane's angles of the per-cell sums of the reduced absorption and
//            scattering systems;
//   reduce   the partial sums across the cell's lanes (LDS, fixed order);
//   solve    the quartic in T' (FP64 Newton) and the 2 x 2 scattering system,
//            redundantly in every lane of the cell;
//   phase C  I^{n+1}_m from the per-angle values kept in registers since
//            phase B, written once; partial moments, reduced like the sums.
//
// The per-interface data that do not change within a call (alpha, the
// interface flow speed, the IV Courant factor) come from a table built once
// per call by k_faces; 3 v J per cell (IV = n . wv) comes with the moments.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rt_common.hpp"

namespace rtk {

constexpr int kNmomX = 13;  // moments (10) + wv = 3 v J (3)
constexpr int kNsum = 22;   // per-cell sums of phase B

struct Step2Args {
  int ndim, n[3], ncell, nang;
  int bc[3][2];
  int stride[3];
  double dt, C, invC, P, cvfac;
  double dt_dx[3];
  double dl10[3];
  double vol, rtol;
  int maxit, estimate_v;
  const double *mu;      // [3][nang]
  const double *w;       // [nang]
  const double *ghost;   // [3][2][nang]
  const double *sa, *ss, *rho, *v;
  double *T;
  const double *faces;   // [3][3][ncell]: alpha, hv, u of the low face of each cell
  const double *mom_in;  // [13][ncell] E, F, P, wv of I^n
  double *mom_out;       // [13][ncell] of I^{n+1}
  double *oE, *oF, *oP;
  double *dEgas, *dMom;
  int accumulate;
  double *partials;
  int *status;
  const void *I_in;
  void *I_out;
  const void *dF_in;
  void *dF_out;
};

// ----------------------------------------------------------- arithmetic
// Reciprocal: hardware estimate refined by Newton steps (two in FP64, none
// beyond the hardware's in FP32); differs from a correctly rounded divide by
// at most an ulp.
__device__ __forceinline__ double fast_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  return r;
}
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

template <typename A>
__device__ __forceinline__ A vl_face(A up2, A up1, A dn1, A h) {
  // up1 + h * vanLeer(up1 - up2, dn1 - up1), vanLeer(a,b) = 2ab/(a+b) if ab > 0
  const A a = up1 - up2, b = dn1 - up1;
  const A ab = a * b;
  const A q = (ab + ab) * fast_rcp(a + b);
  return up1 + h * (ab > A(0) ? q : A(0));
}

// ----------------------------------------------------------- reductions
// Sums R values over the SLOTS lanes of every cell of the block, in a fixed
// order; every lane of a cell receives the totals.  buf needs
// CPB * R * SLOTS doubles and tot CPB * R doubles of shared memory.
template <int SLOTS, int R>
__device__ __forceinline__ void cell_reduce(double (&x)[R], double *buf, double *tot, int cl,
                                            int slot) {
#pragma unroll
  for (int r = 0; r < R; ++r) buf[(cl * R + r) * SLOTS + slot] = x[r];
  __syncthreads();
  for (int r = slot; r < R; r += SLOTS) {
    const double *p = buf + (cl * R + r) * SLOTS;
    double s = p[0];
#pragma unroll
    for (int j = 1; j < SLOTS; ++j) s += p[j];
    tot[cl * R + r] = s;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; ++r) x[r] = tot[cl * R + r];
}

// ------------------------------------------------------------ kernels
// Interface table and IV basis.  faces[(d*3 + j)*ncell + c] for the face
// between the cell below c along axis d (wrapped, or the edge cell itself at
// a non-periodic low boundary) and c: j = 0 alpha, 1 hv = (1 - |u| dt/dx)/2,
// 2 u.  wv = 3 v E/(4pi) into mom[10..12].
__global__ __launch_bounds__(kBlock) void k_faces(Step2Args p, double *faces, double *mom) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
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
    faces[(size_t)(d * 3 + 0) * N + c] = alpha_of(sig, p.dl10[d]);
    faces[(size_t)(d * 3 + 1) * N + c] = 0.5 * (1.0 - fabs(u) * p.dt_dx[d]);
    faces[(size_t)(d * 3 + 2) * N + c] = u;
  }
  const double J = mom[c] * (1.0 / kFourPi);
  for (int k = 0; k < 3; ++k) mom[(size_t)(10 + k) * N + c] = 3.0 * p.v[(size_t)k * N + c] * J;
}

// Moments of I (and wv) for the cell-major layout.
template <typename S, int SLOTS>
__global__ __launch_bounds__(kBlock) void k_moments2(Step2Args p) {
  constexpr int CPB = kBlock / SLOTS;
  __shared__ double buf[CPB * 10 * SLOTS];
  __shared__ double tot[CPB * 10];
  const int cl = threadIdx.x / SLOTS, slot = threadIdx.x % SLOTS;
  const int c = blockIdx.x * CPB + cl;
  const bool act = c < p.ncell;
  const S *I = static_cast<const S *>(p.I_in);
  double a[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (act)
    for (int m = slot; m < p.nang; m += SLOTS) {
      const double n0 = p.mu[m], n1 = p.mu[p.nang + m], n2 = p.mu[2 * p.nang + m];
      const double Iw = double(I[(size_t)c * p.nang + m]) * p.w[m];
      a[0] += Iw;
      a[1] += n0 * Iw;
      a[2] += n1 * Iw;
      a[3] += n2 * Iw;
      a[4] += n0 * n0 * Iw;
      a[5] += n1 * n1 * Iw;
      a[6] += n2 * n2 * Iw;
      a[7] += n0 * n1 * Iw;
      a[8] += n0 * n2 * Iw;
      a[9] += n1 * n2 * Iw;
    }
  cell_reduce<SLOTS, 10>(a, buf, tot, cl, slot);
  if (!act) return;
  const size_t N = (size_t)p.ncell;
  for (int k = slot; k < 10; k += SLOTS) p.mom_out[(size_t)k * N + c] = kFourPi * a[k];
  if (slot == 0) {
    if (p.oE) p.oE[c] = kFourPi * a[0];
    if (p.oF)
      for (int k = 0; k < 3; ++k) p.oF[(size_t)k * N + c] = kFourPi * a[1 + k];
    if (p.oP)
      for (int k = 0; k < 6; ++k) p.oP[(size_t)k * N + c] = kFourPi * a[4 + k];
  }
}

// Per-cell, per-axis stencil data (uniform over the lanes of a cell).
template <typename A>
struct Stencil {
  int idx[4];      // cells at offsets -2, -1, +1, +2 along the axis
  int kind[4];     // 0 read, 1 fixed table, 2 vacuum
  A wv[4][3];      // 3 v J at those cells
  A aL, aR, hL, hR;
  double uL, uR;
};

template <typename A, bool PER>
__device__ __forceinline__ void load_stencil(const Step2Args &p, int c, const int q[3], int d,
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
        kk = k < 0 ? k + n : k - n;
        if (kk < 0 || kk >= n) kk = ((k % n) + n) % n;
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
  s.uL = p.faces[(size_t)(d * 3 + 2) * N + c];
  if (PER || q[d] + 1 < n || p.bc[d][1] == kPeriodic) {
    const int cr = s.idx[2];
    s.aR = A(p.faces[(size_t)(d * 3 + 0) * N + cr]);
    s.hR = A(p.faces[(size_t)(d * 3 + 1) * N + cr]);
    s.uR = p.faces[(size_t)(d * 3 + 2) * N + cr];
  } else {
    // high non-periodic boundary: the ghost copies this cell's fields
    const double sig = p.sa[c] + p.ss[c];
    const double u = p.v[(size_t)d * N + c];
    s.aR = A(alpha_of(sig, p.dl10[d]));
    s.hR = A(0.5 * (1.0 - fabs(u) * p.dt_dx[d]));
    s.uR = u;
  }
}

template <typename S, typename A, bool PER>
__device__ __forceinline__ A ghost_load(const Step2Args &p, const S *I, int idx, int kind,
                                        int side, int d, int m, A mud) {
  const size_t at = (size_t)idx * p.nang + m;
  if (PER || kind == 0) return A(I[at]);
  if (kind == 1) return A(p.ghost[(size_t)(d * 2 + side) * p.nang + m]);
  const bool outgoing = side == 0 ? (mud < A(0)) : (mud > A(0));
  return outgoing ? A(I[at]) : A(0);
}

template <typename S, typename A, int SLOTS, int KMAX, bool PER, bool FUSED>
__global__ __launch_bounds__(kBlock) void k_step2(Step2Args p) {
  constexpr int CPB = kBlock / SLOTS;
  __shared__ double red_buf[CPB * kNsum * SLOTS];
  __shared__ double red_tot[CPB * kNsum];
  const int cl = threadIdx.x / SLOTS, slot = threadIdx.x % SLOTS;
  const int c0 = blockIdx.x * CPB + cl;
  const bool act = c0 < p.ncell;
  const int c = act ? c0 : p.ncell - 1;  // inactive lanes shadow the last cell
  const int NA = p.nang;
  const size_t N = (size_t)p.ncell;
  const S *Iin = static_cast<const S *>(p.I_in);
  S *Iout = static_cast<S *>(p.I_out);
  const double C = p.C, P = p.P, dt = p.dt;
  const double sa = p.sa[c], ss = p.ss[c], rho = p.rho[c], Tn = p.T[c];
  const double v0 = p.v[c], v1 = p.v[N + c], v2 = p.v[2 * N + c];

  // ------------------------------------------------ phase A: transport
  A Ic[KMAX], dF[KMAX];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    const int m = slot + SLOTS * k;
    Ic[k] = m < NA ? A(Iin[(size_t)c * NA + m]) : A(0);
    dF[k] = A(0);
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
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        const int m = slot + SLOTS * k;
        if (m >= NA) break;
        const A n0 = A(p.mu[m]), n1 = A(p.mu[NA + m]), n2 = A(p.mu[2 * NA + m]);
        const A mud = d == 0 ? n0 : d == 1 ? n1 : n2;
        if (mud == A(0)) continue;
        const bool up = mud > A(0);
        A IV[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) IV[j] = n0 * s.wv[j][0] + n1 * s.wv[j][1] + n2 * s.wv[j][2];
        const A IVc = n0 * wc0 + n1 * wc1 + n2 * wc2;
        const A Itc = Ic[k] - IVc * invC;
        const A Im1 = ghost_load<S, A, PER>(p, Iin, s.idx[1], s.kind[1], 0, d, m, mud);
        const A Ip1 = ghost_load<S, A, PER>(p, Iin, s.idx[2], s.kind[2], 1, d, m, mud);
        const A Ifar = ghost_load<S, A, PER>(p, Iin, up ? s.idx[0] : s.idx[3],
                                             up ? s.kind[0] : s.kind[3], up ? 0 : 1, d, m, mud);
        const A Itm1 = Im1 - IV[1] * invC, Itp1 = Ip1 - IV[2] * invC;
        const A Itfar = Ifar - (up ? IV[0] : IV[3]) * invC;
        const A h = A(0.5) * (A(1) - AC * fabs(mud) * dtdx);
        // upwind frame: U1 upwind neighbour, U2 the one behind it, D1 downwind
        const A U1 = up ? Itm1 : Itp1, D1 = up ? Itp1 : Itm1;
        const A fout = vl_face(U1, Itc, D1, h);    // face downwind of the cell
        const A fin = vl_face(Itfar, U1, Itc, h);  // face upwind of the cell
        const A upR = up ? fout : fin, upL = up ? fin : fout;
        const A cenR = A(0.5) * (Itc + Itp1), cenL = A(0.5) * (Itm1 + Itc);
        const A phiR = AC * mud * (s.aR * upR + (A(1) - s.aR) * cenR);
        const A phiL = AC * mud * (s.aL * upL + (A(1) - s.aL) * cenL);
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
        dF[k] -= dtdx * ((phiR + mud * ivR) - (phiL + mud * ivL));
      }
    }
  } else {
    const S *dFin = static_cast<const S *>(p.dF_in);
    if (dFin) {
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        const int m = slot + SLOTS * k;
        if (m < NA) dF[k] = A(dFin[(size_t)c * NA + m]);
      }
    }
  }

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
  A pk[KMAX], Ak[KMAX], Bk[KMAX];
  A sum[kNsum];
#pragma unroll
  for (int r = 0; r < kNsum; ++r) sum[r] = A(0);
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    const int m = slot + SLOTS * k;
    pk[k] = A(0);
    Ak[k] = A(0);
    Bk[k] = A(0);
    if (m >= NA) continue;
    const A n0 = A(p.mu[m]), n1 = A(p.mu[NA + m]), n2 = A(p.mu[2 * NA + m]);
    const A Wm = A(p.w[m]);
    const A t = n0 * Au0 + n1 * Au1 + n2 * Au2;
    const A D = D0 - dsa * t, aw = AW0 - dss * t;
    const A rDa = fast_rcp(D * aw);
    const A invD = aw * rDa, invaw = D * rDa;
    const A e = E0 + A(3) * dsa * t;
    const A g = Auu + t * t;
    const A b = B0 + A(2) * dss * t - dssC * t * t;
    const A cm = A(-3) * dss * t;
    const A r4 = to5 ? Ic[k] : Ic[k] + dF[k];
    const A pm = r4 * invD + (to5 ? dF[k] : A(0));
    pk[k] = pm;
    Ak[k] = invaw;
    Bk[k] = invD * invaw;
    const A WD = Wm * invD, Wa = Wm * invaw, Wad = Wa * invD;
    sum[0] += WD * r4;
    sum[1] += WD * e;
    sum[2] += WD;
    sum[3] += WD * t * r4;
    sum[4] += WD * t * e;
    sum[5] += WD * t;
    sum[6] += WD * g * r4;
    sum[7] += WD * g * e;
    sum[8] += WD * g;
    sum[9] += Wa * b * pm;
    sum[10] += Wa * pm;
    sum[11] += Wa * b;
    sum[12] += Wa * b * cm;
    sum[13] += Wa;
    sum[14] += Wa * cm;
    sum[15] += Wad * b * e;
    sum[16] += Wad * b;
    sum[17] += Wad * e;
    sum[18] += Wad;
    const A WI = Wm * (Ic[k] + dF[k]);
    sum[19] += n0 * WI;
    sum[20] += n1 * WI;
    sum[21] += n2 * WI;
  }
  double Sm[kNsum];
#pragma unroll
  for (int r = 0; r < kNsum; ++r) Sm[r] = double(sum[r]);
  cell_reduce<SLOTS, kNsum>(Sm, red_buf, red_tot, cl, slot);

  // --------------------------------------------- solve (FP64, per cell)
  const double kap = dt * sa / C;
  const double qden = 1.0 + kap * Sm[8];
  const double q0 = Sm[6] / qden, q1 = Sm[7] / qden;
  const double j0 = Sm[0] - kap * Sm[2] * q0, j1 = Sm[1] - kap * Sm[2] * q1;
  const double k0 = Sm[3] - kap * Sm[5] * q0, k1 = Sm[4] - kap * Sm[5] * q1;
  const double beta = P * C * (1.0 - uu / (C * C)) * sa * dt;
  const double g8 = 8.0 * kPi * P * sa * dt;
  const double h0 = -g8 * (k0 - q0 / C) + kFourPi * beta * j0;
  const double h1q = (-g8 * (k1 - q1 / C) - kFourPi * beta * (1.0 - j1)) * (1.0 / kFourPi);
  const double cv = rho * p.cvfac;
  double T = Tn;
  int it = 0;
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
  if (act && slot == 0 && (!conv || !(T > 0.0) || !isfinite(T))) atomicOr(p.status, 1);
  const double X = T * T * T * T * (1.0 / kFourPi);
  const double Q = q0 + q1 * X;
  const double Sbr = Sm[9] + X * Sm[15] - kap * Q * Sm[16];
  const double Sr5 = Sm[10] + X * Sm[17] - kap * Q * Sm[18];
  const double a11 = 1.0 + Sm[11], a12 = Sm[12], a21 = Sm[13], a22 = 1.0 + Sm[14];
  const double det = a11 * a22 - a12 * a21;
  const double s1 = (Sbr * a22 - a12 * Sr5) / det;
  const double s2 = (a11 * Sr5 - a21 * Sbr) / det;

  // --------------------------------------- phase C: new intensities
  const A AX = A(X), AkQ = A(kap * Q), As1 = A(s1), As2 = A(s2);
  double mo[11];
#pragma unroll
  for (int r = 0; r < 10; ++r) mo[r] = 0.0;
  mo[10] = 1.0e300;
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    const int m = slot + SLOTS * k;
    if (m >= NA) break;
    const double d0 = p.mu[m], d1 = p.mu[NA + m], d2 = p.mu[2 * NA + m];
    const A t = A(d0) * Au0 + A(d1) * Au1 + A(d2) * Au2;
    const A e = E0 + A(3) * dsa * t;
    const A cm = A(-3) * dss * t;
    const S Inew = S(Ak[k] * (pk[k] - As1 - cm * As2) + Bk[k] * (e * AX - AkQ));
    if (act) Iout[(size_t)c * NA + m] = Inew;
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
  {
    // sums and the minimum share one pass through shared memory
    double tmp[10];
#pragma unroll
    for (int r = 0; r < 10; ++r) tmp[r] = mo[r];
    cell_reduce<SLOTS, 10>(tmp, red_buf, red_tot, cl, slot);
    double mn = mo[10];
#pragma unroll
    for (int o = 1; o < SLOTS; o <<= 1) mn = fmin(mn, __shfl_xor(mn, o, 64));
#pragma unroll
    for (int r = 0; r < 10; ++r) mo[r] = tmp[r] * kFourPi;
    mo[10] = mn;
  }

  // ------------------------------------------------ Step 7 and outputs
  const double f4 = kFourPi * P / C;
  const double dm0 = -(P / C) * mo[1] + f4 * Sm[19];
  const double dm1 = -(P / C) * mo[2] + f4 * Sm[20];
  const double dm2 = -(P / C) * mo[3] + f4 * Sm[21];
  const double m0 = rho * v0, m1 = rho * v1, m2 = rho * v2;
  const double ek = (((m0 + dm0) * (m0 + dm0) + (m1 + dm1) * (m1 + dm1) + (m2 + dm2) * (m2 + dm2)) -
                     (m0 * m0 + m1 * m1 + m2 * m2)) /
                    (2.0 * rho);
  const double deg = cv * (T - Tn) + ek;
  if (act) {
    // per-cell stores spread over the lanes of the cell
    const double J1 = mo[0] * (1.0 / kFourPi);
    for (int f = slot; f < 18; f += SLOTS) {
      double val;
      double *dst;
      if (f < 10) {
        val = mo[f];
        dst = p.mom_out + (size_t)f * N;
      } else if (f < 13) {
        const double vk = f == 10 ? v0 : f == 11 ? v1 : v2;
        val = 3.0 * vk * J1;
        dst = p.mom_out + (size_t)f * N;
      } else if (f == 13) {
        val = T;
        dst = p.T;
      } else if (f == 14) {
        if (!p.dEgas) continue;
        val = (p.accumulate ? p.dEgas[c] : 0.0) + deg;
        dst = p.dEgas;
      } else {
        if (!p.dMom) continue;
        const int k = f - 15;
        const double dm = k == 0 ? dm0 : k == 1 ? dm1 : dm2;
        val = (p.accumulate ? p.dMom[(size_t)k * N + c] : 0.0) + dm;
        dst = p.dMom + (size_t)k * N;
      }
      dst[c] = val;
    }
    if (slot == 0) {
      if (p.oE) p.oE[c] = mo[0];
      if (p.oF)
        for (int k = 0; k < 3; ++k) p.oF[(size_t)k * N + c] = mo[1 + k];
      if (p.oP)
        for (int k = 0; k < 6; ++k) p.oP[(size_t)k * N + c] = mo[4 + k];
    }
  }
  double tot[kNtot];
#pragma unroll
  for (int k = 0; k < kNtot; ++k) tot[k] = 0.0;
  tot[10] = 1.0e300;
  if (act && slot == 0) {
    const double vol = p.vol;
    tot[0] = P * mo[0] * vol;
    tot[1] = cv * T * vol;
    tot[2] = deg * vol;
    tot[3] = ek * vol;
    tot[4] = dm0 * vol;
    tot[5] = dm1 * vol;
    tot[6] = dm2 * vol;
    tot[7] = P / C * mo[1] * vol;
    tot[8] = P / C * mo[2] * vol;
    tot[9] = P / C * mo[3] * vol;
    tot[10] = mo[10];
    tot[11] = double(it);
  }
  block_totals(tot, p.partials);
}

// Transport increment alone (unfused path), cell-major dF.
template <typename S, typename A, int SLOTS, int KMAX, bool PER>
__global__ __launch_bounds__(kBlock) void k_transport2(Step2Args p) {
  constexpr int CPB = kBlock / SLOTS;
  const int cl = threadIdx.x / SLOTS, slot = threadIdx.x % SLOTS;
  const int c = blockIdx.x * CPB + cl;
  if (c >= p.ncell) return;
  const int NA = p.nang;
  const size_t N = (size_t)p.ncell;
  const S *Iin = static_cast<const S *>(p.I_in);
  S *dFo = static_cast<S *>(p.dF_out);
  const int q[3] = {c % p.n[0], (c / p.n[0]) % p.n[1], c / (p.n[0] * p.n[1])};
  const A wc0 = A(p.mom_in[10 * N + c]), wc1 = A(p.mom_in[11 * N + c]),
          wc2 = A(p.mom_in[12 * N + c]);
  const A AC = A(p.C), invC = A(p.invC);
  A Ic[KMAX], dF[KMAX];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    const int m = slot + SLOTS * k;
    Ic[k] = m < NA ? A(Iin[(size_t)c * NA + m]) : A(0);
    dF[k] = A(0);
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (d >= p.ndim) break;
    Stencil<A> s;
    load_stencil<A, PER>(p, c, q, d, s);
    const A dtdx = A(p.dt_dx[d]);
    const bool posR = s.uR > 0.0, posL = s.uL > 0.0;
    const bool zeroR = s.uR == 0.0, zeroL = s.uL == 0.0;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      const int m = slot + SLOTS * k;
      if (m >= NA) break;
      const A n0 = A(p.mu[m]), n1 = A(p.mu[NA + m]), n2 = A(p.mu[2 * NA + m]);
      const A mud = d == 0 ? n0 : d == 1 ? n1 : n2;
      if (mud == A(0)) continue;
      const bool up = mud > A(0);
      A IV[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) IV[j] = n0 * s.wv[j][0] + n1 * s.wv[j][1] + n2 * s.wv[j][2];
      const A IVc = n0 * wc0 + n1 * wc1 + n2 * wc2;
      const A Itc = Ic[k] - IVc * invC;
      const A Im1 = ghost_load<S, A, PER>(p, Iin, s.idx[1], s.kind[1], 0, d, m, mud);
      const A Ip1 = ghost_load<S, A, PER>(p, Iin, s.idx[2], s.kind[2], 1, d, m, mud);
      const A Ifar = ghost_load<S, A, PER>(p, Iin, up ? s.idx[0] : s.idx[3],
                                           up ? s.kind[0] : s.kind[3], up ? 0 : 1, d, m, mud);
      const A Itm1 = Im1 - IV[1] * invC, Itp1 = Ip1 - IV[2] * invC;
      const A Itfar = Ifar - (up ? IV[0] : IV[3]) * invC;
      const A h = A(0.5) * (A(1) - AC * fabs(mud) * dtdx);
      const A U1 = up ? Itm1 : Itp1, D1 = up ? Itp1 : Itm1;
      const A fout = vl_face(U1, Itc, D1, h);
      const A fin = vl_face(Itfar, U1, Itc, h);
      const A upR = up ? fout : fin, upL = up ? fin : fout;
      const A cenR = A(0.5) * (Itc + Itp1), cenL = A(0.5) * (Itm1 + Itc);
      const A phiR = AC * mud * (s.aR * upR + (A(1) - s.aR) * cenR);
      const A phiL = AC * mud * (s.aL * upL + (A(1) - s.aL) * cenL);
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
      dF[k] -= dtdx * ((phiR + mud * ivR) - (phiL + mud * ivL));
    }
  }
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    const int m = slot + SLOTS * k;
    if (m < NA) dFo[(size_t)c * NA + m] = S(dF[k]);
  }
}

}  // namespace rtk
