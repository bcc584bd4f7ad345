// Thread-per-cell step kernels (angle-major layout I[m][c]): one lane owns a
// cell and loops over all its angles, with a uniform angle across the wave.
// Two passes over the angles: pass 1 computes the transport increment and
// the per-cell sums of the reduced absorption / scattering systems and
// stages p_m in the output buffer; pass 2 forms I^{n+1}.  Used for every
// angle count (the fused step for sets larger than the wave-group kernel
// handles), and for the moments and the transport-only entry point.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rt_common.hpp"

namespace rtk {

// --------------------------------------------------------- neighbourhood
// Per-cell transport context: the four neighbours along each active axis
// (offsets -2, -1, +1, +2), their field data, and the interface data.
template <typename A>
struct Axis {
  int idx[4];       // cell to read (wrapped when periodic, edge cell otherwise)
  int kind[4];      // 0 read idx, 1 fixed table, 2 vacuum (read if outgoing)
  A wv[4][3];       // 3 v J at the neighbours (IV = n . wv)
  A alphaL, alphaR; // transport speed factors of the faces j-1/2, j+1/2
  double uL, uR;    // interface flow speeds along the axis
  A hvL, hvR;       // (1 - |u| dt/dx)/2 for the IV interface values
};

template <typename A, bool PER>
__device__ __forceinline__ void build_axis(const StepArgs &p, int c, const int q[3], int d,
                                           const A wc[3], double sigc, double vdc,
                                           Axis<A> &ax) {
  const int n = p.n[d];
  const int offs[4] = {-2, -1, 1, 2};
  double sig[4], vd[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int k = q[d] + offs[j];
    int kk = k, kind = 0;
    if (k < 0 || k >= n) {
      const int side = k < 0 ? 0 : 1;
      const int bc = PER ? kPeriodic : p.bc[d][side];
      if (bc == kPeriodic) {
        kk = ((k % n) + n) % n;
      } else {
        kk = k < 0 ? 0 : n - 1;
        kind = bc == kFixed ? 1 : bc == kVacuum ? 2 : 0;
      }
    }
    const int cj = c + (kk - q[d]) * p.stride[d];
    ax.idx[j] = cj;
    ax.kind[j] = kind;
    const double Jj = p.mom_in[cj] * (1.0 / kFourPi);
    const double vx = p.v[cj], vy = p.v[(size_t)p.ncell + cj], vz = p.v[2 * (size_t)p.ncell + cj];
    ax.wv[j][0] = A(p.ivfac * vx * Jj);
    ax.wv[j][1] = A(p.ivfac * vy * Jj);
    ax.wv[j][2] = A(p.ivfac * vz * Jj);
    sig[j] = p.sa[cj] + p.ss[cj];
    vd[j] = p.v[(size_t)d * p.ncell + cj];
  }
  ax.alphaL = A(alpha_of(0.5 * (sig[1] + sigc), p.dl10[d]));
  ax.alphaR = A(alpha_of(0.5 * (sigc + sig[2]), p.dl10[d]));
  ax.uL = 0.5 * (vd[1] + vdc);
  ax.uR = 0.5 * (vdc + vd[2]);
  ax.hvL = A(0.5 * (1.0 - fabs(ax.uL) * p.dt_dx[d]));
  ax.hvR = A(0.5 * (1.0 - fabs(ax.uR) * p.dt_dx[d]));
  (void)wc;
}

template <typename S, typename A, bool PER>
__device__ __forceinline__ A load_I(const StepArgs &p, const S *Im, const Axis<A> &ax, int j,
                                    int d, int m, A mud) {
  if (PER || ax.kind[j] == 0) return A(Im[ax.idx[j]]);
  const int side = j < 2 ? 0 : 1;
  if (ax.kind[j] == 1) return A(fixed_ghost(p, d, side, m, ax.idx[j]));
  const bool outgoing = side == 0 ? (mud < A(0)) : (mud > A(0));
  return outgoing ? A(Im[ax.idx[j]]) : A(0);
}

// Transport increment of angle m for the cell (Section 4.2): unsplit sum
// over axes of the divergence of the interface fluxes
//   Phi = C mu [alpha I~*_up + (1 - alpha) I~_c] + mu IV*,  I~ = I - IV/C.
template <typename S, typename A, bool PER>
__device__ __forceinline__ A transport_dF(const StepArgs &p, const S *Im, int m, A Ic,
                                          const A wc[3], const Axis<A> (&ax)[3]) {
  const A n0 = A(p.mu[m]), n1 = A(p.mu[p.nang + m]), n2 = A(p.mu[2 * p.nang + m]);
  const A C = A(p.C), invC = A(p.invC);
  const A IVc = n0 * wc[0] + n1 * wc[1] + n2 * wc[2];
  const A Itc = Ic - IVc * invC;
  A dF = A(0);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (d >= p.ndim) break;
    const A mud = d == 0 ? n0 : d == 1 ? n1 : n2;
    if (mud == A(0)) continue;
    const Axis<A> &a = ax[d];
    A IV[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) IV[j] = n0 * a.wv[j][0] + n1 * a.wv[j][1] + n2 * a.wv[j][2];
    const A Im1 = load_I<S, A, PER>(p, Im, a, 1, d, m, mud);
    const A Ip1 = load_I<S, A, PER>(p, Im, a, 2, d, m, mud);
    const A Itm1 = Im1 - IV[1] * invC, Itp1 = Ip1 - IV[2] * invC;
    const A h = A(0.5) * (A(1) - C * fabs(mud) * A(p.dt_dx[d]));
    A upR, upL;
    if (mud > A(0)) {
      const A Im2 = load_I<S, A, PER>(p, Im, a, 0, d, m, mud);
      const A Itm2 = Im2 - IV[0] * invC;
      upR = upwind_face(Itm1, Itc, Itp1, h);
      upL = upwind_face(Itm2, Itm1, Itc, h);
    } else {
      const A Ip2 = load_I<S, A, PER>(p, Im, a, 3, d, m, mud);
      const A Itp2 = Ip2 - IV[3] * invC;
      upR = upwind_face(Itp2, Itp1, Itc, h);
      upL = upwind_face(Itp1, Itc, Itm1, h);
    }
    const A cenR = A(0.5) * (Itc + Itp1), cenL = A(0.5) * (Itm1 + Itc);
    const A phiR = C * mud * (a.alphaR * upR + (A(1) - a.alphaR) * cenR);
    const A phiL = C * mud * (a.alphaL * upL + (A(1) - a.alphaL) * cenL);
    // IV interface values, upwinded by the interface flow speed
    A ivR, ivL;
    {
      const bool pos = a.uR > 0.0;
      const A up2 = pos ? IV[1] : IV[3], up1 = pos ? IVc : IV[2], dn1 = pos ? IV[2] : IVc;
      const A f = upwind_face(up2, up1, dn1, a.hvR);
      ivR = a.uR == 0.0 ? A(0.5) * (IVc + IV[2]) : f;
    }
    {
      const bool pos = a.uL > 0.0;
      const A up2 = pos ? IV[0] : IV[2], up1 = pos ? IV[1] : IVc, dn1 = pos ? IVc : IV[1];
      const A f = upwind_face(up2, up1, dn1, a.hvL);
      ivL = a.uL == 0.0 ? A(0.5) * (IV[1] + IVc) : f;
    }
    dF -= A(p.dt_dx[d]) * ((phiR + mud * ivR) - (phiL + mud * ivL));
  }
  return dF;
}

// Per-cell data shared by the transport and source parts.
template <typename A>
struct CellCtx {
  int q[3];
  A wc[3];
  Axis<A> ax[3];
};

template <typename A, bool PER>
__device__ __forceinline__ void build_cell(const StepArgs &p, int c, CellCtx<A> &cc) {
  cc.q[0] = c % p.n[0];
  cc.q[1] = (c / p.n[0]) % p.n[1];
  cc.q[2] = c / (p.n[0] * p.n[1]);
  const double Jc = p.mom_in[c] * (1.0 / kFourPi);
  const double vc[3] = {p.v[c], p.v[(size_t)p.ncell + c], p.v[2 * (size_t)p.ncell + c]};
#pragma unroll
  for (int k = 0; k < 3; ++k) cc.wc[k] = A(p.ivfac * vc[k] * Jc);
  const double sigc = p.sa[c] + p.ss[c];
#pragma unroll
  for (int d = 0; d < 3; ++d)
    if (d < p.ndim) build_axis<A, PER>(p, c, cc.q, d, cc.wc, sigc, vc[d], cc.ax[d]);
}

// ------------------------------------------------------------- kernels
template <typename S>
__global__ __launch_bounds__(kBlock) void k_moments(StepArgs p) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= p.ncell) return;
  const S *I = static_cast<const S *>(p.I_in);
  double acc[kNmom] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int m = 0; m < p.nang; ++m) {
    const double n0 = p.mu[m], n1 = p.mu[p.nang + m], n2 = p.mu[2 * p.nang + m];
    const double Iw = double(I[(size_t)m * p.ncell + c]) * p.w[m];
    acc[0] += Iw;
    acc[1] += n0 * Iw;
    acc[2] += n1 * Iw;
    acc[3] += n2 * Iw;
    acc[4] += n0 * n0 * Iw;
    acc[5] += n1 * n1 * Iw;
    acc[6] += n2 * n2 * Iw;
    acc[7] += n0 * n1 * Iw;
    acc[8] += n0 * n2 * Iw;
    acc[9] += n1 * n2 * Iw;
  }
#pragma unroll
  for (int k = 0; k < kNmom; ++k) p.mom_out[(size_t)k * p.ncell + c] = kFourPi * acc[k];
  if (p.oE) p.oE[c] = kFourPi * acc[0];
  if (p.oF)
    for (int k = 0; k < 3; ++k) p.oF[(size_t)k * p.ncell + c] = kFourPi * acc[1 + k];
  if (p.oP)
    for (int k = 0; k < 6; ++k) p.oP[(size_t)k * p.ncell + c] = kFourPi * acc[4 + k];
}

template <typename S, typename A, bool PER>
__global__ __launch_bounds__(kBlock) void k_transport(StepArgs p) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= p.ncell) return;
  CellCtx<A> cc;
  build_cell<A, PER>(p, c, cc);
  const S *I = static_cast<const S *>(p.I_in);
  S *dF = static_cast<S *>(p.dF_out);
  for (int m = 0; m < p.nang; ++m) {
    const S *Im = I + (size_t)m * p.ncell;
    const A Ic = A(Im[c]);
    dF[(size_t)m * p.ncell + c] = S(transport_dF<S, A, PER>(p, Im, m, Ic, cc.wc, cc.ax));
  }
}

// Temperature of the reduced absorption system (Section 4.3) from its
// per-cell angle sums at velocity u (uu = u.u): the quartic
// c_v (T - T^n) = h0 + h1 T^4/4pi by Newton from T^n.  Returns T and sets
// X = T^4/4pi, Q = q0 + q1 X, the iteration count and convergence.
struct AbsSums {
  double Sr, Se, S1, Rr, Re, R1, Ar, Ae, A1;
};
__device__ __forceinline__ double abs_solve(const StepArgs &p, const AbsSums &a, double uu,
                                            double sa, double cv, double Tn, double &X,
                                            double &Q, int &it, bool &conv) {
  const double C = p.C, P = p.P, dt = p.dt;
  const double kap = dt * sa / C;
  const double qden = 1.0 + kap * a.A1;
  const double q0 = a.Ar / qden, q1 = a.Ae / qden;
  const double j0 = a.Sr - kap * a.S1 * q0, j1 = a.Se - kap * a.S1 * q1;
  const double k0 = a.Rr - kap * a.R1 * q0, k1 = a.Re - kap * a.R1 * q1;
  const double beta = P * C * (1.0 - uu / (C * C)) * sa * dt;
  const double g8 = 8.0 * kPi * P * sa * dt;
  const double h0 = -g8 * (k0 - q0 / C) + kFourPi * beta * j0;
  const double h1 = -g8 * (k1 - q1 / C) - kFourPi * beta * (1.0 - j1);
  const double h1q = h1 * (1.0 / kFourPi);
  double T = Tn;
  conv = false;
  for (it = 1; it <= p.maxit; ++it) {
    const double T3 = T * T * T;
    const double f = cv * (T - Tn) - h0 - h1q * T3 * T;
    const double fp = cv - 4.0 * h1q * T3;
    const double dT = f / fp;
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

// Fused step (FUSED) or source-only step reading dF_in (!FUSED).
// SO: second order in time for the absorption step (Section 4.3 names
// solving the absorption system twice): the system is solved at the step's
// velocity u, the Step 4 momentum change d4 of that solution gives the
// time-centred velocity uc = v^n + d4/(2 rho), and the system is solved
// again at uc from the same right-hand side and T^n.  The scattering step
// keeps u.  Pass 1 then stages the right-hand side (r4, or dF when dF is
// routed to Step 5) instead of p_m, and pass 1b forms the sums of the second
// solve and of the scattering step.
template <typename S, typename A, bool PER, bool FUSED, bool SO>
__global__ __launch_bounds__(kBlock) void k_step(StepArgs p) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  const bool active = c < p.ncell;
  double tot[kNtot];
#pragma unroll
  for (int k = 0; k < kNtot; ++k) tot[k] = 0.0;
  tot[10] = 1.0e300;

  if (active) {
    const S *Iin = static_cast<const S *>(p.I_in);
    S *Iout = static_cast<S *>(p.I_out);
    const S *dFin = static_cast<const S *>(p.dF_in);
    const double C = p.C, P = p.P, dt = p.dt;
    const double sa = p.sa[c], ss = p.ss[c], rho = p.rho[c], Tn = p.T[c];
    const double v0 = p.v[c], v1 = p.v[(size_t)p.ncell + c], v2 = p.v[2 * (size_t)p.ncell + c];
    const size_t N = (size_t)p.ncell;

    CellCtx<A> cc;
    if (FUSED) build_cell<A, PER>(p, c, cc);

    // Step 3: half-step velocity estimate from the moments of I^n.
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
    const bool to5 = ss > sa;  // Step 2 routing of dF

    // per-angle coefficient pieces (arith type); their reciprocals come from
    // fast_rcp, within an ulp of a divide
    const A Au0 = A(u0), Au1 = A(u1), Au2 = A(u2), Auu = A(uu);
    const A dsa = A(dt * sa), dss = A(dt * ss);
    const A D0 = A(1.0 + dt * sa * C);          // D_m = D0 - dsa t
    const A E0 = A(dt * sa * C);                // e_m = E0 + 3 dsa t
    const A AW0 = A(1.0 + dt * C * ss);         // a_m W_m = AW0 - dss t
    const A B0 = A(-dt * C * ss - dt * ss * uu / C);  // b_m = B0 + 2 dss t - (dss/C) t^2
    const A dssC = A(dt * ss / C);

    // pass 1 accumulators (double)
    AbsSums ab{0, 0, 0, 0, 0, 0, 0, 0, 0};
    double Bp = 0, Pp = 0, Bb = 0, Bc = 0, B1 = 0, Bcc = 0, Be = 0, Bd = 0, Ee = 0, Ed = 0;
    double M0 = 0, M1 = 0, M2 = 0;
    // SO: the Step 4 momentum change of the first solution from
    // I'_m - r4_m = (-dt sa (C - t) r4_m + e_m X - kappa Q)/D_m:
    // sum W n (-dt sa (C - t) r4)/D, sum W n e/D, sum W n/D
    const A AC = A(C);
    double Hd[3] = {0, 0, 0}, He[3] = {0, 0, 0}, H1[3] = {0, 0, 0};

    for (int m = 0; m < p.nang; ++m) {
      const S *Im = Iin + (size_t)m * N;
      const A n0 = A(p.mu[m]), n1 = A(p.mu[p.nang + m]), n2 = A(p.mu[2 * p.nang + m]);
      const A Wm = A(p.w[m]);
      const A Ic = A(Im[c]);
      A dF;
      if (FUSED)
        dF = transport_dF<S, A, PER>(p, Im, m, Ic, cc.wc, cc.ax);
      else
        dF = dFin ? A(dFin[(size_t)m * N + c]) : A(0);
      const A t = n0 * Au0 + n1 * Au1 + n2 * Au2;
      const A invD = fast_rcp(D0 - dsa * t);
      const A e = E0 + A(3) * dsa * t;
      const A g = Auu + t * t;
      const A r4 = to5 ? Ic : Ic + dF;
      const A WD = Wm * invD;
      ab.Sr += double(WD * r4);
      ab.Se += double(WD * e);
      ab.S1 += double(WD);
      ab.Rr += double(WD * t * r4);
      ab.Re += double(WD * t * e);
      ab.R1 += double(WD * t);
      ab.Ar += double(WD * g * r4);
      ab.Ae += double(WD * g * e);
      ab.A1 += double(WD * g);
      const A WI = Wm * (Ic + dF);
      M0 += double(n0 * WI);
      M1 += double(n1 * WI);
      M2 += double(n2 * WI);
      if constexpr (SO) {
        Iout[(size_t)m * N + c] = S(to5 ? dF : r4);
        const double d[3] = {p.mu[m], p.mu[p.nang + m], p.mu[2 * p.nang + m]};
        const double wd = double(WD), wr = double(-(WD * dsa * (AC - t) * r4)),
                     we = double(WD * e);
        for (int k = 0; k < 3; ++k) {
          Hd[k] += d[k] * wr;
          He[k] += d[k] * we;
          H1[k] += d[k] * wd;
        }
      } else {
        const A invaw = fast_rcp(AW0 - dss * t);
        const A b = B0 + A(2) * dss * t - dssC * t * t;
        const A cm = A(-3) * dss * t;
        const A pm = r4 * invD + (to5 ? dF : A(0));
        Iout[(size_t)m * N + c] = S(pm);
        const A Wa = Wm * invaw;
        const A Wad = Wa * invD;
        Bp += double(Wa * b * pm);
        Pp += double(Wa * pm);
        Bb += double(Wa * b);
        Bc += double(Wa * b * cm);
        B1 += double(Wa);
        Bcc += double(Wa * cm);
        Be += double(Wad * b * e);
        Bd += double(Wad * b);
        Ee += double(Wad * e);
        Ed += double(Wad);
      }
    }

    // Step 4: scalar quartic in T' (FP64)
    const double kap = dt * sa / C;
    const double cv = rho * p.cvfac;
    double X, Q;
    int it;
    bool conv;
    double T = abs_solve(p, ab, uu, sa, cv, Tn, X, Q, it, conv);
    // absorption at the time-centred velocity (SO), else at u
    double ua0 = u0, ua1 = u1, ua2 = u2;
    if constexpr (SO) {
      // Step 4 momentum change of the first solution, as the gas sees it
      const double fm = -p.gasfac * kFourPi * P / C;
      ua0 = v0 + fm * (Hd[0] + X * He[0] - kap * Q * H1[0]) / (2.0 * rho);
      ua1 = v1 + fm * (Hd[1] + X * He[1] - kap * Q * H1[1]) / (2.0 * rho);
      ua2 = v2 + fm * (Hd[2] + X * He[2] - kap * Q * H1[2]) / (2.0 * rho);
      const double uua = ua0 * ua0 + ua1 * ua1 + ua2 * ua2;
      const A Ua0 = A(ua0), Ua1 = A(ua1), Ua2 = A(ua2), Auua = A(uua);
      AbsSums a2{0, 0, 0, 0, 0, 0, 0, 0, 0};
      // pass 1b: the sums of the second solve and of the scattering step
      for (int m = 0; m < p.nang; ++m) {
        const size_t at = (size_t)m * N + c;
        const A n0 = A(p.mu[m]), n1 = A(p.mu[p.nang + m]), n2 = A(p.mu[2 * p.nang + m]);
        const A Wm = A(p.w[m]);
        const A q = A(Iout[at]);
        const A r4 = to5 ? A(Iin[at]) : q;
        const A ta = n0 * Ua0 + n1 * Ua1 + n2 * Ua2;
        const A invD = fast_rcp(D0 - dsa * ta);
        const A e = E0 + A(3) * dsa * ta;
        const A g = Auua + ta * ta;
        const A WD = Wm * invD;
        a2.Sr += double(WD * r4);
        a2.Se += double(WD * e);
        a2.S1 += double(WD);
        a2.Rr += double(WD * ta * r4);
        a2.Re += double(WD * ta * e);
        a2.R1 += double(WD * ta);
        a2.Ar += double(WD * g * r4);
        a2.Ae += double(WD * g * e);
        a2.A1 += double(WD * g);
        const A t = n0 * Au0 + n1 * Au1 + n2 * Au2;
        const A invaw = fast_rcp(AW0 - dss * t);
        const A b = B0 + A(2) * dss * t - dssC * t * t;
        const A cm = A(-3) * dss * t;
        const A pm = r4 * invD + (to5 ? q : A(0));
        Iout[at] = S(pm);
        const A Wa = Wm * invaw;
        const A Wad = Wa * invD;
        Bp += double(Wa * b * pm);
        Pp += double(Wa * pm);
        Bb += double(Wa * b);
        Bc += double(Wa * b * cm);
        B1 += double(Wa);
        Bcc += double(Wa * cm);
        Be += double(Wad * b * e);
        Bd += double(Wad * b);
        Ee += double(Wad * e);
        Ed += double(Wad);
      }
      int it2;
      bool conv2;
      T = abs_solve(p, a2, uua, sa, cv, Tn, X, Q, it2, conv2);
      it = it2 > it ? it2 : it;
      conv = conv && conv2;
    }
    if (!conv || !(T > 0.0) || !isfinite(T)) atomicOr(p.status, 1);

    // Step 5: the 2 x 2 system of the scattering step
    const double Sbr = Bp + X * Be - kap * Q * Bd;
    const double Sr5 = Pp + X * Ee - kap * Q * Ed;
    const double a11 = 1.0 + Bb, a12 = Bc, a21 = B1, a22 = 1.0 + Bcc;
    const double det = a11 * a22 - a12 * a21;
    const double s1 = (Sbr * a22 - a12 * Sr5) / det;
    const double s2 = (a11 * Sr5 - a21 * Sbr) / det;

    // pass 2: new intensities and their moments
    const A AX = A(X), AkQ = A(kap * Q), As1 = A(s1), As2 = A(s2);
    const A Ua0 = A(ua0), Ua1 = A(ua1), Ua2 = A(ua2);
    double mom[kNmom] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    double imin = 1.0e300;
    for (int m = 0; m < p.nang; ++m) {
      const A n0 = A(p.mu[m]), n1 = A(p.mu[p.nang + m]), n2 = A(p.mu[2 * p.nang + m]);
      const A t = n0 * Au0 + n1 * Au1 + n2 * Au2;
      const A ta = SO ? n0 * Ua0 + n1 * Ua1 + n2 * Ua2 : t;
      const A invD = fast_rcp(D0 - dsa * ta);
      const A e = E0 + A(3) * dsa * ta;
      const A invaw = fast_rcp(AW0 - dss * t);
      const A cm = A(-3) * dss * t;
      const size_t at = (size_t)m * N + c;
      const A pm = A(Iout[at]);
      const A r5 = pm + (e * AX - AkQ) * invD;
      const S Inew = S((r5 - As1 - cm * As2) * invaw);
      Iout[at] = Inew;
      const double Iw = double(Inew) * p.w[m];
      const double d0 = p.mu[m], d1 = p.mu[p.nang + m], d2 = p.mu[2 * p.nang + m];
      mom[0] += Iw;
      mom[1] += d0 * Iw;
      mom[2] += d1 * Iw;
      mom[3] += d2 * Iw;
      mom[4] += d0 * d0 * Iw;
      mom[5] += d1 * d1 * Iw;
      mom[6] += d2 * d2 * Iw;
      mom[7] += d0 * d1 * Iw;
      mom[8] += d0 * d2 * Iw;
      mom[9] += d1 * d2 * Iw;
      imin = fmin(imin, double(Inew));
    }
#pragma unroll
    for (int k = 0; k < kNmom; ++k) {
      mom[k] *= kFourPi;
      p.mom_out[(size_t)k * N + c] = mom[k];
    }
    if (p.oE) p.oE[c] = mom[0];
    if (p.oF)
      for (int k = 0; k < 3; ++k) p.oF[(size_t)k * N + c] = mom[1 + k];
    if (p.oP)
      for (int k = 0; k < 6; ++k) p.oP[(size_t)k * N + c] = mom[4 + k];

    // Step 7 source terms: momentum from photon momentum conservation,
    // kinetic energy from the fixed gas velocity, internal energy from T'.
    // (gasfac: C over the reduced speed of light, 1 without one)
    const double f4 = kFourPi * P / C, gf = p.gasfac;
    const double dm0 = gf * (-(P / C) * mom[1] + f4 * M0);
    const double dm1 = gf * (-(P / C) * mom[2] + f4 * M1);
    const double dm2 = gf * (-(P / C) * mom[3] + f4 * M2);
    const double m0 = rho * v0, m1 = rho * v1, m2 = rho * v2;
    const double ek = (((m0 + dm0) * (m0 + dm0) + (m1 + dm1) * (m1 + dm1) + (m2 + dm2) * (m2 + dm2)) -
                       (m0 * m0 + m1 * m1 + m2 * m2)) /
                      (2.0 * rho);
    const double dET = cv * gf * (T - Tn);
    const double deg = dET + ek;
    p.T[c] = T;
    if (p.dEgas) p.dEgas[c] = (p.accumulate ? p.dEgas[c] : 0.0) + deg;
    if (p.dMom) {
      p.dMom[c] = (p.accumulate ? p.dMom[c] : 0.0) + dm0;
      p.dMom[N + c] = (p.accumulate ? p.dMom[N + c] : 0.0) + dm1;
      p.dMom[2 * N + c] = (p.accumulate ? p.dMom[2 * N + c] : 0.0) + dm2;
    }
    const double vol = p.vol;
    tot[0] = P * mom[0] * vol;
    tot[1] = cv * gf * T * vol;
    tot[2] = deg * vol;
    tot[3] = ek * vol;
    tot[4] = dm0 * vol;
    tot[5] = dm1 * vol;
    tot[6] = dm2 * vol;
    tot[7] = P / C * mom[1] * vol;
    tot[8] = P / C * mom[2] * vol;
    tot[9] = P / C * mom[3] * vol;
    tot[10] = imin;
    tot[11] = double(it);
  }
  block_totals(tot, p.partials, p.nparts, p.accumulate);
}

}  // namespace rtk
