// Shared device helpers of the radiative-transfer kernels: constants, the
// reduced transport speed factor alpha (Section 4.2), deterministic wave and
// block reductions, and the reduction of per-block partial totals.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rtk {

constexpr int kBlock = 256;
constexpr int kNtot = 12;
constexpr int kNmom = 10;  // E, F(3), P(6)
constexpr double kFourPi = 12.566370614359172953850573533118;
constexpr double kPi = 3.1415926535897932384626433832795;

enum BcKind : int { kPeriodic = 0, kFixed = 1, kCopy = 2, kVacuum = 3 };
constexpr int kNmomX = 13;  // moments (10) + 3 v J (3)
constexpr int kMaxWaves = 8;  // waves per block of the wave-group kernel

// Entries of a per-angle record (StepArgs::arec).
enum RecField : int {
  rec_n0 = 0, rec_n1, rec_n2,   // direction cosines
  rec_h0, rec_h1, rec_h2,       // 1 - C |mu_d| dt/dx_d, d = 0..2
  rec_w,                        // weight
  rec_wn0, rec_wn1, rec_wn2,    // w n_d
  rec_wnn,                      // 6 values: w n_x n_x, w n_y n_y, w n_z n_z, w n_x n_y, w n_x n_z, w n_y n_z
  rec_flags = rec_wnn + 6,      // integer bits in the slot: bit d n_d > 0, bit 3 + d n_d != 0
  kRec = 17
};

// Arguments of every step kernel (passed by value).
struct StepArgs {
  int ndim, n[3], ncell, nang;
  int bc[3][2];
  int stride[3];
  double dt, C, invC, P, cvfac;  // cvfac = R/(gamma - 1) (times c_r/C, below)
  double gasfac;                 // C/c_r: gas change per radiation change (1 at c_r = C)
  double dt_dx[3];               // dt / dx_d
  double dl10[3];                // 10 dx_d (transport speed factor alpha; 0 gives alpha = 1)
  double ivfac;                  // 3 in IV = 3 n.v J (0: no IV split, I~ = I)
  double vol, rtol;
  int maxit, estimate_v;
  const double *mu;      // [3][nang]
  const double *w;       // [nang]
  const float *muf;      // FP32 copies of mu and w (FP32 arithmetic)
  const float *wf;
  // per call, one record of kRec values per angle (padded with zero records
  // to the slots of the wave-group kernel): the direction, the Courant
  // factors 1 - C |mu_d| dt/dx_d of the slope terms, and the quadrature
  // weights of the moments (layout in rec_*)
  const double *arec;
  const float *arecf;
  const double *ghost;   // [3][2][nang] fixed-face ghost intensities
  const double *gface[6];  // per face (axis*2 + side): [nang][ncell / n[axis]]
                           // position-dependent ghosts of a fixed face, or null
  const double *sa, *ss, *rho;
  double *v;             // [3][ncell]; written only with feedback
  int feedback;          // gas feedback: v <- v + d(rho v)/rho after the step
  double *T;
  const double *faces;   // [3][3][ncell] of the low face of each cell: C alpha, the
                         // lower cell's share of the centred IV value, signed 1 - nu_v
  const double *mom_in;  // [13][ncell] E, F(3), P(6), 3vJ(3) of I^n
  double *mom_out;       // [13][ncell] of I^{n+1}
  double *oE, *oF, *oP;  // optional copies of the new moments
  double *dEgas, *dMom;  // optional per-cell sums over the call
  int accumulate;
  double *partials;      // [kNtot][nparts] per-block partial totals
  int nparts;            // rows of partials: blocks (tiles of cells) of the launch
  int *status;
  const void *I_in;
  void *I_out;
  const void *dF_in;     // unfused source step: transport increment (nullable)
  void *dF_out;          // transport-only output
};

// ----------------------------------------------------------------- helpers
// Reciprocal from the hardware estimate refined by Newton steps (two in
// FP64; the FP32 estimate is used as is).  Within an ulp of a divide.
__device__ __forceinline__ double fast_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  return r;
}
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Reciprocal of the limiter: in FP64 one Newton step on the hardware
// estimate (relative error about the square of the estimate's, some tens of
// ulp).  It only scales the slope correction of an interface value, never an
// intensity itself; the source steps keep fast_rcp.  One step instead of two
// on the twelve limiters of a cell-angle measured 3 % faster in the fused
// step kernel.
__device__ __forceinline__ double limiter_rcp(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float limiter_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// van Leer harmonic-mean slope of the one-sided differences (zero at
// extrema), and the upwind interface value of the piecewise-linear
// reconstruction at Courant number nu, with h = (1 - nu)/2.
template <typename A>
__device__ __forceinline__ A van_leer(A a, A b) {
  const A ab = a * b;
  return ab > A(0) ? (A(2) * ab) * limiter_rcp(a + b) : A(0);
}
template <typename A>
__device__ __forceinline__ A upwind_face(A up2, A up1, A dn1, A h) {
  return up1 + h * van_leer(up1 - up2, dn1 - up1);
}

// alpha = sqrt((1 - exp(-tau))/tau), tau = (10 dl sigma)^2, alpha(0) = 1
// Ghost intensity of angle m beside edge cell e of the fixed face (d, side):
// from the face's position-dependent table when it has one (face cells in
// order of the two other axes, lower axis fastest), else from its angle
// table.  Both ghost layers take the value.
__device__ __forceinline__ double fixed_ghost(const StepArgs &p, int d, int side, int m, int e) {
  const double *f = p.gface[d * 2 + side];
  if (!f) return p.ghost[(size_t)(d * 2 + side) * p.nang + m];
  const int n0 = p.n[0], n01 = p.n[0] * p.n[1];
  const int fi = d == 0 ? e / n0 : d == 1 ? e % n0 + n0 * (e / n01) : e % n01;
  return f[(size_t)m * (size_t)(p.ncell / p.n[d]) + fi];
}

// The IV value of the face between a lower cell L and an upper cell U
// (Section 4.2: IV is advected at the flow speed u of the face, upwinded by
// the sign of u, centred at u = 0), written as
//   IV* = l IV_L + (1 - l) IV_U + f q_up,
// with l = 1 (u > 0), 0 (u < 0) or 1/2 (u = 0), f = sign(u) (1 - |u| dt/dx)
// and q_up half the van Leer slope of the upwind cell.
__device__ __forceinline__ double iv_lower_share(double u) {
  return u > 0.0 ? 1.0 : (u < 0.0 ? 0.0 : 0.5);
}
__device__ __forceinline__ double iv_signed_factor(double u, double dt_dx) {
  const double h = 1.0 - fabs(u) * dt_dx;
  return u > 0.0 ? h : (u < 0.0 ? -h : 0.0);
}

__device__ __forceinline__ double alpha_of(double sigma, double dl10) {
  const double s = dl10 * sigma;
  const double tau = s * s;
  return tau > 0.0 ? sqrt(-expm1(-tau) / tau) : 1.0;
}

// Blocks are dispatched round-robin over the eight XCDs (block b runs on XCD
// b % 8, each with its own L2).  Renumbering them so that every XCD works
// through one contiguous range of blocks keeps the stencil neighbours of a
// block (the rows and planes next to it) in the same L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb / 8;
  if (b >= 8 * q) return b;
  return (b % 8) * q + b / 8;
}

// Tile of block b for stencil reuse in L2: each XCD takes a contiguous slab
// of nz/8 z-planes, and inside its slab the z-planes vary fastest, so that
// the tiles above, below, in front and behind a tile (its stencil
// neighbours along y and z) run on the same XCD within a few tens of blocks
// of it.  Grids whose planes do not hold whole tiles, or with fewer than 8
// planes, take the XCD-contiguous order.
// With sub > 0 (dividing the slab depth) the slab is worked through in
// sub-slabs of sub planes, so that the tiles beside a tile along y are nearer
// in time, at the price of the z-neighbours across sub-slab boundaries.
__device__ __forceinline__ int slab_block(int b, int nb, const int (&n)[3], int sub = 0) {
  const int plane = n[0] * n[1];
  if (n[2] < 8 || (n[2] & 7) || (plane & 63)) return xcd_block(b, nb);
  const int pt = plane >> 6;           // tiles per z-plane
  const int zc = n[2] >> 3;            // z-planes per XCD slab
  const int pos = (b & 7) * (nb >> 3) + (b >> 3);
  const int slab = pos / (zc * pt), r = pos - slab * (zc * pt);
  if (sub > 0 && sub < zc && zc % sub == 0) {
    const int ss = r / (sub * pt), r2 = r - ss * (sub * pt);
    return (slab * zc + ss * sub + r2 % sub) * pt + r2 / sub;
  }
  const int z = slab * zc + r % zc;
  return z * pt + r / zc;
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}
__device__ __forceinline__ double wave_min(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmin(x, __shfl_xor(x, o, 64));
  return x;
}
__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
  return x;
}

// Stores a block's totals of one step into its row b of the partials
// [kNtot][nparts]: the exchange sums (entries 2..6) add to the row's value
// from the earlier steps of the call, entry 11 keeps the maximum, the state
// entries are overwritten.  accumulate = 0 on the first step of a call.
// The rows are reduced once, after the last step of the call.
__device__ __forceinline__ void store_partial(double *partials, int nparts, int b, int k, double x,
                                              int accumulate) {
  double *dst = partials + (size_t)k * nparts + b;
  if (accumulate) {
    if (k >= 2 && k <= 6)
      x = *dst + x;
    else if (k == 11)
      x = fmax(*dst, x);
  }
  *dst = x;
}

// Deterministic per-block reduction of the totals vector into partials.
__device__ __forceinline__ void block_totals(double (&t)[kNtot], double *partials, int nparts,
                                             int accumulate) {
  __shared__ double red[kBlock / 64][kNtot];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kNtot; ++k) {
    double x = t[k];
    x = (k == 10) ? wave_min(x) : (k == 11) ? wave_max(x) : wave_sum(x);
    if (lane == 0) red[wid][k] = x;
  }
  __syncthreads();
  if (threadIdx.x < kNtot) {
    const int k = threadIdx.x;
    double x = red[0][k];
    for (int q = 1; q < kBlock / 64; ++q)
      x = (k == 10) ? fmin(x, red[q][k]) : (k == 11) ? fmax(x, red[q][k]) : x + red[q][k];
    store_partial(partials, nparts, blockIdx.x, k, x, accumulate);
  }
}

// Deterministic reduction of the per-block partial totals [kNtot][nb] by
// one block of any size that is a multiple of 64 (up to 1024 threads).  The
// rows are dealt to kVLanes virtual lanes (row b to lane b % kVLanes); each
// virtual lane adds its rows in order, each virtual wave of 64 lanes is
// reduced by the same shuffle tree, and the kVLanes / 64 wave results are
// added in order, so the result does not depend on the block size.  out
// receives the kNtot totals.  red: kNtot * (kVLanes / 64) doubles of LDS.
constexpr int kVLanes = 1024;
constexpr int kVWaves = kVLanes / 64;

__device__ __forceinline__ double tot_op(int k, double x, double y) {
  return k == 10 ? fmin(x, y) : k == 11 ? fmax(x, y) : x + y;
}
__device__ __forceinline__ double tot_init(int k) { return k == 10 ? 1.0e300 : 0.0; }

__device__ __forceinline__ void totals_reduce(const double *partials, int nb, double *out,
                                              double *red) {
  const int lane = threadIdx.x & 63;
  for (int vw = threadIdx.x >> 6; vw < kVWaves; vw += blockDim.x >> 6) {
    const int vl = vw * 64 + lane;
    double x[kNtot];
#pragma unroll
    for (int k = 0; k < kNtot; ++k) x[k] = tot_init(k);
    for (int b = vl; b < nb; b += kVLanes) {
#pragma unroll
      for (int k = 0; k < kNtot; ++k) x[k] = tot_op(k, x[k], partials[(size_t)k * nb + b]);
    }
#pragma unroll
    for (int k = 0; k < kNtot; ++k) {
      const double y = k == 10 ? wave_min(x[k]) : k == 11 ? wave_max(x[k]) : wave_sum(x[k]);
      if (lane == 0) red[k * kVWaves + vw] = y;
    }
  }
  __syncthreads();
  if (threadIdx.x < kNtot) {
    const int k = threadIdx.x;
    double x = red[k * kVWaves];
    for (int q = 1; q < kVWaves; ++q) x = tot_op(k, x, red[k * kVWaves + q]);
    out[k] = x;
  }
  __syncthreads();
}

}  // namespace rtk
