// icr_device.hpp -- device-side pieces of the heliospheric MHD update for
// CDNA4 (gfx950): state conversions (Eq. 6, mu0 = 1), fast speeds, the
// physical flux of Eqs. (1)-(4), slope limiters, the TVDLF/HLL face flux and
// the cell-centred source terms (spherical geometry, gravity, centrifugal
// and Coriolis force of the co-rotating frame, Sect. 2).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace icr {

constexpr int NV = 8;  // rho, m_r, m_t, m_p, e, B_r, B_t, B_p

enum : int { FLUX_TVDLF = 0, FLUX_HLL = 1, FLUX_HLLD = 2 };
enum : int { LIM_MINMOD = 0, LIM_MC = 1, LIM_WENO5 = 2 };  // WENO5: 3 ghost layers

constexpr int BAD_NONE = 0x7fffffff;

// Device-resident clock and step control.  Written by the last block of the
// stage-2 kernel (or the CFL kernel) and by the begin-of-call kernel; read
// by every kernel of a step so that no host round trip is needed.
struct DevClock {
  double t;        // current time (code units)
  double dt;       // dt of the next step (clipped to t_end)
  double dt_cfl;   // CFL dt of the next step before clipping
  double t_end;    // <= 0: no end time
  double last_dt;  // dt of the last completed step
  double resid;    // last ||rho^{n+1} - rho^n|| / ||rho^n||
  long long step;  // completed steps
  long long taken; // steps completed in the current icr_step call
  int active;      // 1: the next step advances the state
  int clip;        // 1: the next step ends exactly at t_end
  int bad;         // first invalid cell index or BAD_NONE
  int advanced;    // 1: a step completed since the probe logger last ran
  unsigned int counter;  // arrival counter of the last-block reduction
  int pad0;
  long long n_log;       // probe records written
  long long last_sample; // floor(t / cadence) of the last probe record
};

// Metric factors of one precision (see k_metric for definitions).
template <typename R>
struct Metric {
  const R *rm2, *rp2, *ivr, *hr, *gr, *irc, *grav, *idr, *rc;  // per r cell
  const R *sm, *sp, *ict, *cot, *snc, *csc, *phf, *ilph;  // per theta cell
  R ilth;                                                 // 1 / dtheta
};

// Element idx of a device array: a 32-bit byte offset from a wave-uniform
// base (the grid setup keeps every array below 4 GiB).  Loads of several
// arrays at the same index then share one offset register instead of each
// holding a 64-bit address.
template <typename T>
__device__ __forceinline__ T ldg(const T* base, unsigned idx) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) +
                                     idx * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void stg(T* base, unsigned idx, T x) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + idx * (unsigned)sizeof(T)) = x;
}

// Reflecting colatitude edges: a row index beyond [0, nt) reads the mirror
// row (-1 - j below, 2 nt - 1 - j above, clamped to the grid) with the theta
// components of velocity and field negated (flip = true).
__device__ __forceinline__ int mirror_row(int j, int nt, bool& flip) {
  flip = j < 0 || j >= nt;
  const int m = j < 0 ? -1 - j : (j >= nt ? 2 * nt - 1 - j : j);
  return m < 0 ? 0 : (m >= nt ? nt - 1 : m);
}

template <typename R>
__device__ __forceinline__ void flip_theta(R (&w)[NV]) {
  w[2] = -w[2];
  w[6] = -w[6];
}

template <typename R>
__device__ __forceinline__ R rmax(R a, R b) { return a > b ? a : b; }
template <typename R>
__device__ __forceinline__ R rmin(R a, R b) { return a < b ? a : b; }

// Reciprocal and square root for the face-once kernel.  FP64: the hardware
// estimate refined by Newton-Raphson (reciprocal, y <- y + y (1 - x y),
// twice) or by Goldschmidt's coupled iteration for g ~ sqrt(x),
// h ~ 1/(2 sqrt(x)) (twice, then one residual correction); both end within
// about one ulp for normal positive x.  FP32: the single hardware op.
__device__ __forceinline__ double rcp_fast(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, y, 1.0);
  y = __builtin_fma(y, e, y);
  e = __builtin_fma(-x, y, 1.0);
  return __builtin_fma(y, e, y);
}
__device__ __forceinline__ float rcp_fast(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ double sqrt_fast(double x) {  // x > 0
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  double r = __builtin_fma(-g, h, 0.5);
  g = __builtin_fma(g, r, g);
  h = __builtin_fma(h, r, h);
  r = __builtin_fma(-g, h, 0.5);
  g = __builtin_fma(g, r, g);
  h = __builtin_fma(h, r, h);
  const double d = __builtin_fma(-g, g, x);
  return __builtin_fma(d, h, g);
}
__device__ __forceinline__ float sqrt_fast(float x) { return __builtin_amdgcn_sqrtf(x); }

// Smallest positive argument passed to sqrt_fast for a square root that may
// be exactly zero (keeps the estimate finite; far below any resolved value).
template <typename R>
__device__ __forceinline__ R sqrt_floor();
template <>
__device__ __forceinline__ double sqrt_floor<double>() { return 1e-280; }
template <>
__device__ __forceinline__ float sqrt_floor<float>() { return 1e-30f; }

template <typename R, bool FAST = false>
__device__ __forceinline__ void cons2prim(const R (&u)[NV], R (&w)[NV], R gm1) {
  const R rho = u[0];
  const R ir = FAST ? rcp_fast(rho) : R(1) / rho;
  w[0] = rho;
  w[1] = u[1] * ir;
  w[2] = u[2] * ir;
  w[3] = u[3] * ir;
  const R kin = R(0.5) * (u[1] * w[1] + u[2] * w[2] + u[3] * w[3]);
  const R mag = R(0.5) * (u[5] * u[5] + u[6] * u[6] + u[7] * u[7]);
  w[4] = gm1 * (u[4] - kin - mag);
  w[5] = u[5];
  w[6] = u[6];
  w[7] = u[7];
}

template <typename R>
__device__ __forceinline__ void prim2cons(const R (&w)[NV], R (&u)[NV], R igm1) {
  const R rho = w[0];
  u[0] = rho;
  u[1] = rho * w[1];
  u[2] = rho * w[2];
  u[3] = rho * w[3];
  const R kin = R(0.5) * (u[1] * w[1] + u[2] * w[2] + u[3] * w[3]);
  const R mag = R(0.5) * (w[5] * w[5] + w[6] * w[6] + w[7] * w[7]);
  u[4] = w[4] * igm1 + kin + mag;
  u[5] = w[5];
  u[6] = w[6];
  u[7] = w[7];
}

// Fast magnetosonic speed along local component N (1..3):
// c_f^2 = [a^2 + b^2 + sqrt((a^2 + b^2)^2 - 4 a^2 B_n^2 / rho)] / 2.
template <typename R, int N, bool FAST = false>
__device__ __forceinline__ R cfast(const R (&w)[NV], R gam) {
  const R ir = FAST ? rcp_fast(w[0]) : R(1) / w[0];
  const R a2 = gam * w[4] * ir;
  const R b2 = (w[5] * w[5] + w[6] * w[6] + w[7] * w[7]) * ir;
  const R bn = w[4 + N];
  const R s = a2 + b2;
  R disc = s * s - R(4) * a2 * bn * bn * ir;
  if (FAST) {
    // floors keep exact zeros (possible only for invalid states) at ~0
    disc = rmax(disc, sqrt_floor<R>());
    return sqrt_fast(rmax(R(0.5) * (s + sqrt_fast(disc)), sqrt_floor<R>()));
  }
  disc = rmax(disc, R(0));
  return sqrt(R(0.5) * (s + sqrt(disc)));
}

// Physical flux through a face normal to local component N.
template <typename R, int N>
__device__ __forceinline__ void phys_flux(const R (&w)[NV], const R (&u)[NV], R (&f)[NV]) {
  const R vn = w[N], bn = w[4 + N];
  const R ptot = w[4] + R(0.5) * (w[5] * w[5] + w[6] * w[6] + w[7] * w[7]);
  const R vb = w[1] * w[5] + w[2] * w[6] + w[3] * w[7];
  f[0] = w[0] * vn;
#pragma unroll
  for (int d = 1; d <= 3; ++d) f[d] = u[d] * vn - bn * w[4 + d];
  f[N] += ptot;
  f[4] = (u[4] + ptot) * vn - bn * vb;
#pragma unroll
  for (int d = 1; d <= 3; ++d) f[4 + d] = vn * w[4 + d] - bn * w[d];
}

// minmod(a, b): 0 if a b <= 0, else the argument of smaller magnitude.
// MC(a, b): 0 if a b <= 0, else sign(a) min(2|a|, 2|b|, |a + b|/2).
// FAST form: the same functions as max(min(x...), min(max(x...), 0)) over the
// candidate slopes (2a, 2b, (a+b)/2 for MC), which is branch-free.
template <typename R, int LIM, bool FAST = false>
__device__ __forceinline__ R limiter(R a, R b) {
  if (FAST) {
    if (LIM == LIM_MINMOD) return fmax(fmin(a, b), fmin(fmax(a, b), R(0)));
    const R x = R(2) * a, y = R(2) * b, z = R(0.5) * (a + b);
    const R lo = fmin(fmin(x, y), z), hi = fmax(fmax(x, y), z);
    return fmax(lo, fmin(hi, R(0)));
  }
  if (a * b <= R(0)) return R(0);
  if (LIM == LIM_MINMOD) return fabs(a) < fabs(b) ? a : b;
  R m = rmin(R(2) * fabs(a), R(2) * fabs(b));
  m = rmin(m, R(0.5) * fabs(a + b));
  return a > R(0) ? m : -m;
}

// Face states from four consecutive cells (m-2, m-1, m, m+1) around face
// m-1/2: W_L = W_{m-1} + s_{m-1}/2, W_R = W_m - s_m/2, limited undivided
// slopes on primitives.
template <typename R, int LIM, bool FAST = false>
__device__ __forceinline__ void reconstruct(const R (&a)[NV], const R (&b)[NV],
                                            const R (&c)[NV], const R (&d)[NV],
                                            R (&wl)[NV], R (&wr)[NV]) {
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const R db = b[v] - a[v], dc = c[v] - b[v], dd = d[v] - c[v];
    wl[v] = b[v] + R(0.5) * limiter<R, LIM, FAST>(db, dc);
    wr[v] = c[v] - R(0.5) * limiter<R, LIM, FAST>(dc, dd);
  }
}

// WENO5 (Jiang & Shu 1996) value at the face between cells c and d from the
// five cells a..e: the three third-order candidates of the stencils ending
// at, centred on and starting at c, weighted by d_k / (eps + beta_k)^2 with
// linear weights (1, 6, 3)/10 and smoothness indicators beta_k; eps is 1e-6
// of the stencil's mean square (plus 1e-40), so the weights are free of units.
template <typename R, bool FAST = false>
__device__ __forceinline__ R weno5(R a, R b, R c, R d, R e) {
  constexpr R sixth = R(1) / R(6);
  const R q0 = (R(2) * a - R(7) * b + R(11) * c) * sixth;
  const R q1 = (-b + R(5) * c + R(2) * d) * sixth;
  const R q2 = (R(2) * c + R(5) * d - e) * sixth;
  const R s0 = a - R(2) * b + c, t0 = a - R(4) * b + R(3) * c;
  const R s1 = b - R(2) * c + d, t1 = b - d;
  const R s2 = c - R(2) * d + e, t2 = R(3) * c - R(4) * d + e;
  const R b0 = R(13) / R(12) * s0 * s0 + R(0.25) * t0 * t0;
  const R b1 = R(13) / R(12) * s1 * s1 + R(0.25) * t1 * t1;
  const R b2 = R(13) / R(12) * s2 * s2 + R(0.25) * t2 * t2;
  // absolute floor: (floor)^2 must stay a normal number (FP32: 1e-15)
  const R eps = R(1e-6) * (a * a + b * b + c * c + d * d + e * e) * R(0.2) +
                (sizeof(R) == 8 ? R(1e-40) : R(1e-15));
  const R g0 = (eps + b0) * (eps + b0), g1 = (eps + b1) * (eps + b1), g2 = (eps + b2) * (eps + b2);
  if constexpr (sizeof(R) == 8) {
    // weights d_k / g_k scaled by g0 g1 g2: one division (products stay in
    // range in FP64: g >= 1e-80)
    const R a0 = R(0.1) * g1 * g2, a1 = R(0.6) * g0 * g2, a2 = R(0.3) * g0 * g1;
    if constexpr (FAST) return (a0 * q0 + a1 * q1 + a2 * q2) * rcp_fast(a0 + a1 + a2);
    return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
  } else {
    const R a0 = R(0.1) / g0, a1 = R(0.6) / g1, a2 = R(0.3) / g2;
    return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
  }
}

// WENO5 face states of face m-1/2 from the six cells m-3 .. m+2 (p0..p5);
// a face state with rho or p <= 0 falls back to its cell value.
template <typename R, bool FAST = false>
__device__ __forceinline__ void reconstruct_weno5(const R (&p0)[NV], const R (&p1)[NV],
                                                  const R (&p2)[NV], const R (&p3)[NV],
                                                  const R (&p4)[NV], const R (&p5)[NV],
                                                  R (&wl)[NV], R (&wr)[NV]) {
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    wl[v] = weno5<R, FAST>(p0[v], p1[v], p2[v], p3[v], p4[v]);
    wr[v] = weno5<R, FAST>(p5[v], p4[v], p3[v], p2[v], p1[v]);
  }
  if (!(wl[0] > R(0) && wl[4] > R(0)))
#pragma unroll
    for (int v = 0; v < NV; ++v) wl[v] = p2[v];
  if (!(wr[0] > R(0) && wr[4] > R(0)))
#pragma unroll
    for (int v = 0; v < NV; ++v) wr[v] = p3[v];
}

// Numerical flux from the two face states: TVDLF
// F = (F_L + F_R)/2 - alpha (U_R - U_L)/2, alpha = max(|v_n| + c_f), or HLL
// with S_L = min(v_nL - c_fL, v_nR - c_fR), S_R = max(v_nL + c_fL, ...).
// HLLD flux (Miyoshi & Kusano 2005) through a face with normal component N:
// the outer fast waves, the two rotational waves and the contact bound four
// intermediate states sharing the contact speed S_M and total pressure;
// density is continuous across the rotational waves.  Both face states use
// the mean normal field; the normal field's own flux is the HLL value with
// the same outer speeds.
template <typename R, int N, bool FAST>
__device__ __forceinline__ void hlld_flux(const R (&wl0)[NV], const R (&wr0)[NV], R gam, R igm1,
                                          R (&fs)[NV]) {
  constexpr int T1 = N == 1 ? 2 : 1, T2 = N == 3 ? 2 : 3;
  auto rcp = [](R x) { return FAST ? rcp_fast(x) : R(1) / x; };
  const R bn = R(0.5) * (wl0[4 + N] + wr0[4 + N]);
  const R dbn = wr0[4 + N] - wl0[4 + N];
  R w[2][NV], u[2][NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    w[0][v] = wl0[v];
    w[1][v] = wr0[v];
  }
  w[0][4 + N] = bn;
  w[1][4 + N] = bn;
  prim2cons<R>(w[0], u[0], igm1);
  prim2cons<R>(w[1], u[1], igm1);
  const R cmax = rmax(cfast<R, N, FAST>(w[0], gam), cfast<R, N, FAST>(w[1], gam));
  const R sl = rmin(w[0][N], w[1][N]) - cmax, sr = rmax(w[0][N], w[1][N]) + cmax;
  const R fbn = (sl < R(0) && sr > R(0)) ? sl * sr * dbn * rcp(sr - sl) : R(0);
  // every region's flux needs the physical flux of one side only
  if (sl >= R(0) || sr <= R(0)) {
    const bool left = sl >= R(0);
    R wa[NV], ua[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      wa[v] = left ? w[0][v] : w[1][v];
      ua[v] = left ? u[0][v] : u[1][v];
    }
    phys_flux<R, N>(wa, ua, fs);
    fs[4 + N] = fbn;
    return;
  }
  R pt[2], d[2];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    pt[a] = w[a][4] + R(0.5) * (w[a][5] * w[a][5] + w[a][6] * w[a][6] + w[a][7] * w[a][7]);
    d[a] = ((a ? sr : sl) - w[a][N]) * w[a][0];  // mass flux relative to the outer wave
  }
  const R idd = rcp(d[1] - d[0]);
  const R sm = (d[1] * w[1][N] - d[0] * w[0][N] - pt[1] + pt[0]) * idd;
  const R pts = (d[1] * pt[0] - d[0] * pt[1] + d[0] * d[1] * (w[1][N] - w[0][N])) * idd;
  // outer star states of both sides (the double-star state needs both)
  R us[2][NV], sq[2];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const R s = a ? sr : sl;
    const R ism = rcp(s - sm);
    const R rho = d[a] * ism;
    const R den = d[a] * (s - sm) - bn * bn;
    R vt1 = w[a][T1], vt2 = w[a][T2], bt1 = w[a][4 + T1], bt2 = w[a][4 + T2];
    if (fabs(den) > R(1e-12) * (fabs(d[a] * (s - sm)) + bn * bn)) {
      const R iden = rcp(den);
      const R fv = bn * (sm - w[a][N]) * iden;
      const R fb = (d[a] * (s - w[a][N]) - bn * bn) * iden;
      vt1 -= bt1 * fv;
      vt2 -= bt2 * fv;
      bt1 *= fb;
      bt2 *= fb;
    }
    const R vb = w[a][1] * w[a][5] + w[a][2] * w[a][6] + w[a][3] * w[a][7];
    const R vbs = sm * bn + vt1 * bt1 + vt2 * bt2;
    us[a][0] = rho;
    us[a][N] = rho * sm;
    us[a][T1] = rho * vt1;
    us[a][T2] = rho * vt2;
    us[a][4] = ((s - w[a][N]) * u[a][4] - pt[a] * w[a][N] + pts * sm + bn * (vb - vbs)) * ism;
    us[a][4 + N] = bn;
    us[a][4 + T1] = bt1;
    us[a][4 + T2] = bt2;
    sq[a] = FAST ? sqrt_fast(rho) : sqrt(rho);
  }
  // the side of the contact the face lies on: F*_a = F_a + S_a (U*_a - U_a)
  const bool left = sm >= R(0);
  R q[NV], fa[NV];
  {
    R wa[NV], ua[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      wa[v] = left ? w[0][v] : w[1][v];
      ua[v] = left ? u[0][v] : u[1][v];
      q[v] = left ? us[0][v] : us[1][v];
    }
    phys_flux<R, N>(wa, ua, fa);
    const R sa = left ? sl : sr;
#pragma unroll
    for (int v = 0; v < NV; ++v) fa[v] += sa * (q[v] - ua[v]);
  }
  const R ssl = sm - fabs(bn) * rcp(sq[0]), ssr = sm + fabs(bn) * rcp(sq[1]);
  if (ssl >= R(0) || ssr <= R(0)) {
#pragma unroll
    for (int v = 0; v < NV; ++v) fs[v] = fa[v];
    fs[4 + N] = fbn;
    return;
  }
  // double-star state between the rotational waves
  const R sg = bn >= R(0) ? R(1) : R(-1);
  const R isq = rcp(sq[0] + sq[1]);
  const R vl1 = us[0][T1] / us[0][0], vl2 = us[0][T2] / us[0][0];
  const R vr1 = us[1][T1] / us[1][0], vr2 = us[1][T2] / us[1][0];
  const R v1 = (sq[0] * vl1 + sq[1] * vr1 + (us[1][4 + T1] - us[0][4 + T1]) * sg) * isq;
  const R v2 = (sq[0] * vl2 + sq[1] * vr2 + (us[1][4 + T2] - us[0][4 + T2]) * sg) * isq;
  const R b1 = (sq[0] * us[1][4 + T1] + sq[1] * us[0][4 + T1] + sq[0] * sq[1] * (vr1 - vl1) * sg) *
               isq;
  const R b2 = (sq[0] * us[1][4 + T2] + sq[1] * us[0][4 + T2] + sq[0] * sq[1] * (vr2 - vl2) * sg) *
               isq;
  const R vbs = (q[N] * q[4 + N] + q[T1] * q[4 + T1] + q[T2] * q[4 + T2]) / q[0];
  const R vbss = sm * bn + v1 * b1 + v2 * b2;
  R uss[NV];
  uss[0] = q[0];
  uss[N] = q[0] * sm;
  uss[T1] = q[0] * v1;
  uss[T2] = q[0] * v2;
  uss[4] = q[4] + (left ? -sq[0] : sq[1]) * (vbs - vbss) * sg;
  uss[4 + N] = bn;
  uss[4 + T1] = b1;
  uss[4 + T2] = b2;
  const R ssa = left ? ssl : ssr;
#pragma unroll
  for (int v = 0; v < NV; ++v) fs[v] = fa[v] + ssa * (uss[v] - q[v]);
  fs[4 + N] = fbn;
}

template <typename R, int N, int FLUX, bool FAST = false>
__device__ __forceinline__ void face_flux(const R (&wl)[NV], const R (&wr)[NV],
                                          R gam, R igm1, R (&fs)[NV]) {
  if constexpr (FLUX == FLUX_HLLD) {
    hlld_flux<R, N, FAST>(wl, wr, gam, igm1, fs);
    return;
  }
  R ul[NV], ur[NV], fl[NV], fr[NV];
  prim2cons<R>(wl, ul, igm1);
  prim2cons<R>(wr, ur, igm1);
  phys_flux<R, N>(wl, ul, fl);
  phys_flux<R, N>(wr, ur, fr);
  const R cl = cfast<R, N, FAST>(wl, gam), cr = cfast<R, N, FAST>(wr, gam);
  if (FLUX == FLUX_TVDLF) {
    const R alpha = rmax(fabs(wl[N]) + cl, fabs(wr[N]) + cr);
#pragma unroll
    for (int v = 0; v < NV; ++v)
      fs[v] = R(0.5) * (fl[v] + fr[v]) - R(0.5) * alpha * (ur[v] - ul[v]);
  } else {
    const R sl = rmin(wl[N] - cl, wr[N] - cr);
    const R sr = rmax(wl[N] + cl, wr[N] + cr);
    if (sl >= R(0)) {
#pragma unroll
      for (int v = 0; v < NV; ++v) fs[v] = fl[v];
    } else if (sr <= R(0)) {
#pragma unroll
      for (int v = 0; v < NV; ++v) fs[v] = fr[v];
    } else {
      const R id = FAST ? rcp_fast(sr - sl) : R(1) / (sr - sl);
#pragma unroll
      for (int v = 0; v < NV; ++v)
        fs[v] = (sr * fl[v] - sl * fr[v] + sl * sr * (ur[v] - ul[v])) * id;
    }
  }
}

// Cell-centred sources: spherical geometric terms with area-difference
// pressure factors G_r = dA_r/V, H_r*cot(theta_c) = dA_theta/V; gravity
// g = -GM/r^2 e_r (momentum rho g, energy rho v.g); co-rotating frame with
// Omega along the polar axis: F = rho (Omega x r) x Omega + 2 rho v x Omega
// and energy source v.F.
//
// The metric factors of the cell come through an accessor: CellMetric reads
// the global arrays at (i, j); the face-once stage kernel passes one that
// reads its tile's copy in LDS (the same values).
enum MetricR { MR_RM2, MR_RP2, MR_IVR, MR_HR, MR_GR, MR_IRC, MR_GRAV, MR_IDR, MR_RC, MR_N };
enum MetricT { MT_SM, MT_SP, MT_ICT, MT_COT, MT_SNC, MT_CSC, MT_PHF, MT_ILPH, MT_N };

template <typename R>
__device__ __forceinline__ const R* metric_r(const Metric<R>& m, int a) {
  switch (a) {
    case MR_RM2: return m.rm2;
    case MR_RP2: return m.rp2;
    case MR_IVR: return m.ivr;
    case MR_HR: return m.hr;
    case MR_GR: return m.gr;
    case MR_IRC: return m.irc;
    case MR_GRAV: return m.grav;
    case MR_IDR: return m.idr;
    default: return m.rc;
  }
}
template <typename R>
__device__ __forceinline__ const R* metric_t(const Metric<R>& m, int a) {
  switch (a) {
    case MT_SM: return m.sm;
    case MT_SP: return m.sp;
    case MT_ICT: return m.ict;
    case MT_COT: return m.cot;
    case MT_SNC: return m.snc;
    case MT_CSC: return m.csc;
    case MT_PHF: return m.phf;
    default: return m.ilph;
  }
}

template <typename R>
struct CellMetric {
  const Metric<R>& m;
  int i, j;
  __device__ __forceinline__ R r(int a) const { return ldg(metric_r(m, a), (unsigned)i); }
  __device__ __forceinline__ R t(int a) const { return ldg(metric_t(m, a), (unsigned)j); }
  __device__ __forceinline__ R ilth() const { return m.ilth; }
};

template <typename R, typename CM>
__device__ __forceinline__ void add_sources_cm(const R (&w)[NV], const CM& cm, R omega,
                                               int gravity, int corot, R (&L)[NV]) {
  const R rho = w[0], vr = w[1], vt = w[2], vp = w[3], p = w[4];
  const R br = w[5], bt = w[6], bp = w[7];
  const R irc = cm.r(MR_IRC);
  const R cot = cm.t(MT_COT);
  const R ptot = p + R(0.5) * (br * br + bt * bt + bp * bp);
  L[1] += (rho * (vt * vt + vp * vp) - (bt * bt + bp * bp)) * irc + ptot * cm.r(MR_GR);
  L[2] += (-(rho * vr * vt - br * bt) + cot * (rho * vp * vp - bp * bp)) * irc +
          ptot * cm.r(MR_HR) * cot;
  L[3] -= ((rho * vp * vr - bp * br) + cot * (rho * vp * vt - bp * bt)) * irc;
  L[6] += (vr * bt - vt * br) * irc;
  L[7] += ((vr * bp - vp * br) + cot * (vt * bp - vp * bt)) * irc;
  if (gravity) {
    const R g = cm.r(MR_GRAV);
    L[1] += rho * g;
    L[4] += rho * vr * g;
  }
  if (corot) {
    const R sn = cm.t(MT_SNC), cs = cm.t(MT_CSC);
    const R r = cm.r(MR_RC);
    const R cen = rho * omega * omega * r * sn;
    const R cor = R(2) * rho * omega;
    L[1] += cen * sn + cor * vp * sn;
    L[2] += cen * cs + cor * vp * cs;
    L[3] -= cor * (vr * sn + vt * cs);
    L[4] += cen * (vr * sn + vt * cs);
  }
}

template <typename R>
__device__ __forceinline__ void add_sources(const R (&w)[NV], const Metric<R>& m, int i, int j,
                                            R omega, int gravity, int corot, R (&L)[NV]) {
  add_sources_cm<R>(w, CellMetric<R>{m, i, j}, omega, gravity, corot, L);
}

}  // namespace icr
