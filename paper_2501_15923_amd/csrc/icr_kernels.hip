// icr_kernels.hip -- HIP kernels of the heliospheric MHD hot path (gfx950).
//
//   k_metric        per-r / per-theta metric factors of the stretched
//                   spherical grid (radially stretched grid, Sect. 2)
//   k_boundary      inner-boundary primitives at the two RK stage times:
//                   time interpolation between maps (Sect. 3) and the
//                   cone-CME overwrite (Sect. 3.2); one value serves both
//                   ghost layers (Sect. 2.1)
//   k_stage         fused reconstruct + flux + divergence + sources + RK2
//                   combine (Sect. 2 Eqs. 1-6); stage 2 also reduces the
//                   next CFL dt, the relaxation residual and the validity
//                   flag, finishing in its last block
//   k_cfl           CFL dt of the current state (after init / set_state)
//   k_probe_*       trajectory interpolation, frame change and trilinear
//                   sampling on the stretched grid (Sect. 2)
//
// Layouts: state [8][n_phi][n_theta][n_r] (r fastest), ghost primitives
// [8][n_phi][n_theta], maps [n_maps][8][n_theta][n_phi] (code units).
#include "icr_kernels.hpp"

namespace icr {

// ---------------------------------------------------------------- metric --
// r edges r_in q^i; V_r = (r+^3 - r-^3)/3 written as (r+ - r-)(r+^2 + r+ r-
// + r-^2)/3 and G_r = (r+^2 - r-^2)/V_r = 3 (r+ + r-)/(r+^2 + r+ r- + r-^2)
// to avoid cancellation; C_theta = cos t- - cos t+ = 2 sin(t_c) sin(dt/2);
// (sin t+ - sin t-)/C_theta = cot(t_c).
template <typename R>
__global__ void k_metric(MetricArgs a, R* __restrict__ mr) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int nr = a.nr, nt = a.nt;
  double* m64 = a.m64;
  if (t < nr) {
    const int i = t;
    const double rm = a.r_in * pow(a.q, (double)i);
    const double rp = (i + 1 == nr) ? a.r_out : a.r_in * pow(a.q, (double)(i + 1));
    const double s2 = rp * rp + rp * rm + rm * rm;
    const double vr = (rp - rm) * s2 / 3.0;
    const double gr = 3.0 * (rp + rm) / s2;
    const double rc = 0.5 * (rm + rp);
    double v[R_ARRAYS] = {rm * rm, rp * rp, 1.0 / vr, 0.5 * gr, gr, 1.0 / rc,
                          -a.gm / (rc * rc), 1.0 / (rp - rm), rc};
    for (int q = 0; q < R_ARRAYS; ++q) {
      m64[q * nr + i] = v[q];
      mr[q * nr + i] = (R)v[q];
    }
    m64[OFF_REDGE64(nr, nt) + i] = rm;
    if (i + 1 == nr) m64[OFF_REDGE64(nr, nt) + nr] = rp;
  } else if (t < nr + nt) {
    const int j = t - nr;
    const double tm = a.th_min + (a.th_max - a.th_min) * (double)j / nt;
    const double tp = a.th_min + (a.th_max - a.th_min) * (double)(j + 1) / nt;
    const double tc = 0.5 * (tm + tp);
    const double dth = a.th_max - a.th_min;
    const double dt_cell = dth / nt;
    const double sc = sin(tc), cc = cos(tc);
    const double ct = 2.0 * sc * sin(0.5 * (tp - tm));
    double v[T_ARRAYS] = {sin(tm), sin(tp), 1.0 / ct, cc / sc, sc, cc,
                          dt_cell / (ct * a.dph), 1.0 / (sc * a.dph)};
    const int base = R_ARRAYS * nr;
    for (int q = 0; q < T_ARRAYS; ++q) {
      m64[base + q * nt + j] = v[q];
      mr[base + q * nt + j] = (R)v[q];
    }
    m64[OFF_TC64(nr, nt) + j] = tc;
  }
}

template <typename R>
Metric<R> metric_view(const R* base, int nr, int nt, double dth) {
  Metric<R> m;
  const R* p = base;
  m.rm2 = p + 0 * nr; m.rp2 = p + 1 * nr; m.ivr = p + 2 * nr; m.hr = p + 3 * nr;
  m.gr = p + 4 * nr;  m.irc = p + 5 * nr; m.grav = p + 6 * nr; m.idr = p + 7 * nr;
  m.rc = p + 8 * nr;
  const R* q = base + R_ARRAYS * nr;
  m.sm = q + 0 * nt; m.sp = q + 1 * nt; m.ict = q + 2 * nt; m.cot = q + 3 * nt;
  m.snc = q + 4 * nt; m.csc = q + 5 * nt; m.phf = q + 6 * nt; m.ilph = q + 7 * nt;
  m.ilth = (R)(1.0 / dth);
  return m;
}
template Metric<double> metric_view<double>(const double*, int, int, double);
template Metric<float> metric_view<float>(const float*, int, int, double);

void launch_metric(const MetricArgs& a, void* mr, bool f32, hipStream_t s) {
  const int n = a.nr + a.nt;
  if (f32)
    hipLaunchKernelGGL(k_metric<float>, dim3((n + 255) / 256), dim3(256), 0, s, a, (float*)mr);
  else
    hipLaunchKernelGGL(k_metric<double>, dim3((n + 255) / 256), dim3(256), 0, s, a, (double*)mr);
}

// ------------------------------------------------------------- boundary --
// Primitive at the inner shell for column (j, k) at code time t.
__device__ void boundary_prim(const BndArgs& a, double t, int j, int k, double (&w)[NV]) {
  const long long plane = (long long)a.nt * a.np;
  const long long q = (long long)j * a.np + k;
  const int n = a.n_maps;
  if (n == 1 || t <= a.tau[0]) {
    for (int v = 0; v < NV; ++v) w[v] = a.maps[v * plane + q];
  } else if (t >= a.tau[n - 1]) {
    for (int v = 0; v < NV; ++v) w[v] = a.maps[((long long)(n - 1) * NV + v) * plane + q];
  } else {
    int lo = 0, hi = n - 1;  // tau[lo] <= t < tau[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (a.tau[mid] <= t) lo = mid; else hi = mid;
    }
    const double wgt = (t - a.tau[lo]) / (a.tau[lo + 1] - a.tau[lo]);
    for (int v = 0; v < NV; ++v) {
      const double x0 = a.maps[((long long)lo * NV + v) * plane + q];
      const double x1 = a.maps[((long long)(lo + 1) * NV + v) * plane + q];
      w[v] = (1.0 - wgt) * x0 + wgt * x1;
    }
  }
  if (a.n_cme > 0) {
    const double th = a.tc[j];
    const double ph = (k + 0.5) * a.dph;
    const double sth = sin(th), cth = cos(th);
    for (int c = 0; c < a.n_cme; ++c) {
      const double* m = a.cme + 8 * c;  // t0, dur, colat, lon, cos(hw), v, rho, p
      if (!(t >= m[0] && t < m[0] + m[1])) continue;
      const double cosd = cth * cos(m[2]) + sth * sin(m[2]) * cos(ph - m[3]);
      if (cosd >= m[4]) {
        w[0] = m[6];
        w[1] = m[5];
        w[2] = 0.0;
        w[3] = -a.omega * a.r_in * sth;
        w[4] = m[7];
      }
    }
  }
}

template <typename R>
__global__ void k_boundary(BndArgs a, const DevClock* __restrict__ ck, R* __restrict__ g1,
                           R* __restrict__ g2) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int plane = a.nt * a.np;
  if (q >= plane || !ck->active) return;
  const int j = q % a.nt, k = q / a.nt;
  double w[NV];
  boundary_prim(a, ck->t, j, k, w);
  for (int v = 0; v < NV; ++v) g1[(long long)v * plane + q] = (R)w[v];
  boundary_prim(a, ck->t + ck->dt, j, k, w);
  for (int v = 0; v < NV; ++v) g2[(long long)v * plane + q] = (R)w[v];
}

// Boundary at an arbitrary time into a [8][nt][np] double buffer (SI).
__global__ void k_boundary_at(BndArgs a, double t, double* __restrict__ out, Scale sc) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int plane = a.nt * a.np;
  if (q >= plane) return;
  const int j = q / a.np, k = q % a.np;
  double w[NV];
  boundary_prim(a, t, j, k, w);
  for (int v = 0; v < NV; ++v) out[(long long)v * plane + q] = w[v] * sc.s[v];
}

void launch_boundary(const BndArgs& a, const DevClock* ck, void* g1, void* g2, bool f32,
                     hipStream_t s) {
  const int plane = a.nt * a.np;
  const dim3 grid((plane + 255) / 256), blk(256);
  if (f32)
    hipLaunchKernelGGL(k_boundary<float>, grid, blk, 0, s, a, ck, (float*)g1, (float*)g2);
  else
    hipLaunchKernelGGL(k_boundary<double>, grid, blk, 0, s, a, ck, (double*)g1, (double*)g2);
}

void launch_boundary_at(const BndArgs& a, double t, double* out, const Scale& sc, hipStream_t s) {
  const int plane = a.nt * a.np;
  hipLaunchKernelGGL(k_boundary_at, dim3((plane + 255) / 256), dim3(256), 0, s, a, t, out, sc);
}

// ------------------------------------------------------- reductions ------
// Block of 256 threads: max of lam, sums of s1/s0 (fixed tree), min of bad.
__device__ __forceinline__ void block_reduce(double& lam, double& s1, double& s0, int& bad,
                                             double (*sh)[4]) {
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  for (int off = 32; off > 0; off >>= 1) {
    lam = fmax(lam, __shfl_xor(lam, off, 64));
    s1 += __shfl_xor(s1, off, 64);
    s0 += __shfl_xor(s0, off, 64);
    const int ob = __shfl_xor(bad, off, 64);
    bad = ob < bad ? ob : bad;
  }
  const int wv = tid >> 6, lane = tid & 63;
  if (lane == 0) {
    sh[wv][0] = lam;
    sh[wv][1] = s1;
    sh[wv][2] = s0;
    sh[wv][3] = (double)bad;
  }
  __syncthreads();
  if (tid == 0) {
    const int nw = (blockDim.x * blockDim.y) >> 6;
    for (int q = 1; q < nw; ++q) {
      lam = fmax(lam, sh[q][0]);
      s1 += sh[q][1];
      s0 += sh[q][2];
      const int b = (int)sh[q][3];
      bad = b < bad ? b : bad;
    }
  }
}

__device__ void set_next_dt(DevClock* ck, double dtc) {
  ck->dt_cfl = dtc;
  if (ck->t_end > 0.0 && ck->t >= ck->t_end) {
    ck->active = 0;
    ck->dt = 0.0;
    ck->clip = 0;
    return;
  }
  if (ck->t_end > 0.0 && ck->t + dtc >= ck->t_end) {
    ck->dt = ck->t_end - ck->t;
    ck->clip = 1;
  } else {
    ck->dt = dtc;
    ck->clip = 0;
  }
}

// Publish the block partial; the last block to arrive reduces all partials
// in a fixed order and updates the clock.  advance = 1 for the end of an
// RK2 step, 0 for a plain CFL evaluation.
__device__ void finish_reduction(DevClock* ck, double* partials, int nblocks, double cfl,
                                 int advance, double lam, double s1, double s0, int bad) {
  __shared__ double sh[4][4];
  __shared__ int am_last;
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  const int bid = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  block_reduce(lam, s1, s0, bad, sh);
  if (tid == 0) {
    __hip_atomic_store(&partials[4 * bid + 0], lam, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&partials[4 * bid + 1], s1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&partials[4 * bid + 2], s0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&partials[4 * bid + 3], (double)bad, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    const unsigned prev = atomicAdd(&ck->counter, 1u);
    am_last = (prev == (unsigned)(nblocks - 1));
  }
  __syncthreads();
  if (!am_last) return;
  __threadfence();
  double l = 0.0, a1 = 0.0, a0 = 0.0;
  int b = BAD_NONE;
  for (int q = tid; q < nblocks; q += blockDim.x * blockDim.y) {
    l = fmax(l, __hip_atomic_load(&partials[4 * q + 0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    a1 += __hip_atomic_load(&partials[4 * q + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    a0 += __hip_atomic_load(&partials[4 * q + 2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int qb = (int)__hip_atomic_load(&partials[4 * q + 3], __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
    b = qb < b ? qb : b;
  }
  __syncthreads();
  block_reduce(l, a1, a0, b, sh);
  if (tid == 0) {
    if (advance) {
      ck->t = ck->clip ? ck->t_end : ck->t + ck->dt;
      ck->step += 1;
      ck->taken += 1;
      ck->last_dt = ck->dt;
      ck->resid = sqrt(a1) / sqrt(a0);
      ck->advanced = 1;
    }
    if (b != BAD_NONE) {
      if (ck->bad == BAD_NONE || b < ck->bad) ck->bad = b;
      ck->active = 0;
    }
    set_next_dt(ck, cfl / l);
    if (ck->bad != BAD_NONE) ck->active = 0;
    ck->counter = 0;
  }
}

__global__ void k_clock_begin(DevClock* ck, double t_end) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  ck->t_end = t_end;
  ck->taken = 0;
  ck->active = ck->bad == BAD_NONE ? 1 : 0;
  set_next_dt(ck, ck->dt_cfl);
  if (ck->bad != BAD_NONE) ck->active = 0;
}

void launch_clock_begin(DevClock* ck, double t_end, hipStream_t s) {
  hipLaunchKernelGGL(k_clock_begin, dim3(1), dim3(64), 0, s, ck, t_end);
}

// ---------------------------------------------------- stage kernel (v1) --
template <typename R>
__device__ __forceinline__ void load_prim(const StageArgs<R>& a, int i, int j, int k,
                                          R (&w)[NV]) {
  if (i < 0) {
    const long long plane = (long long)a.nt * a.np;
    const long long g = (long long)k * a.nt + j;
#pragma unroll
    for (int v = 0; v < NV; ++v) w[v] = a.ghost[v * plane + g];
    return;
  }
  if (i >= a.nr) i = a.nr - 1;
  const long long c = ((long long)k * a.nt + j) * a.nr + i;
  R u[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = a.uin[v * a.ncell + c];
  cons2prim<R>(u, w, a.gm1);
}

// CFL rate of one cell from its primitives: sum_d (|v_d| + c_f,d) / dx_d.
template <typename R>
__device__ __forceinline__ double cell_rate(const R (&w)[NV], const Metric<R>& m, int i, int j,
                                            R gam) {
  const R lr = (fabs(w[1]) + cfast<R, 1>(w, gam)) * m.idr[i];
  const R lt = (fabs(w[2]) + cfast<R, 2>(w, gam)) * m.irc[i] * m.ilth;
  const R lp = (fabs(w[3]) + cfast<R, 3>(w, gam)) * m.irc[i] * m.ilph[j];
  return (double)(lr + lt + lp);
}

template <typename R>
__device__ __forceinline__ bool cell_valid(const R (&u)[NV], const R (&w)[NV]) {
  bool ok = w[0] > R(0) && w[4] > R(0);
#pragma unroll
  for (int v = 0; v < NV; ++v) ok = ok && isfinite(u[v]);
  return ok;
}

template <typename R, int FLUX, int LIM, int STAGE>
__global__ void __launch_bounds__(256) k_stage_v1(StageArgs<R> a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = blockIdx.z;
  const bool valid = i < a.nr && j < a.nt;
  const int active = a.clock->active;
  const R dt = (R)a.clock->dt;
  double lam = 0.0, s1 = 0.0, s0 = 0.0;
  int bad = BAD_NONE;
  if (valid) {
    const long long c = ((long long)k * a.nt + j) * a.nr + i;
    if (!active) {
      if (STAGE == 2) {
#pragma unroll
        for (int v = 0; v < NV; ++v) a.uout[v * a.ncell + c] = a.un[v * a.ncell + c];
      }
    } else {
      R wc[NV], L[NV];
      load_prim(a, i, j, k, wc);
#pragma unroll
      for (int v = 0; v < NV; ++v) L[v] = R(0);
      {  // r faces i-1/2 and i+1/2
        R w0[NV], w1[NV], w3[NV], w4[NV], wl[NV], wr[NV], fm[NV], fp[NV];
        load_prim(a, i - 2, j, k, w0);
        load_prim(a, i - 1, j, k, w1);
        load_prim(a, i + 1, j, k, w3);
        load_prim(a, i + 2, j, k, w4);
        reconstruct<R, LIM>(w0, w1, wc, w3, wl, wr);
        face_flux<R, 1, FLUX>(wl, wr, a.gam, a.igm1, fm);
        reconstruct<R, LIM>(w1, wc, w3, w4, wl, wr);
        face_flux<R, 1, FLUX>(wl, wr, a.gam, a.igm1, fp);
        const R rm2 = a.m.rm2[i], rp2 = a.m.rp2[i], ivr = a.m.ivr[i];
#pragma unroll
        for (int v = 0; v < NV; ++v) L[v] -= (rp2 * fp[v] - rm2 * fm[v]) * ivr;
      }
      const R hr = a.m.hr[i];
      {  // theta faces, zero-gradient copies beyond the colatitude edges
        R w0[NV], w1[NV], w3[NV], w4[NV], wl[NV], wr[NV], fm[NV], fp[NV];
        const int jm2 = j - 2 < 0 ? 0 : j - 2, jm1 = j - 1 < 0 ? 0 : j - 1;
        const int jp1 = j + 1 >= a.nt ? a.nt - 1 : j + 1;
        const int jp2 = j + 2 >= a.nt ? a.nt - 1 : j + 2;
        load_prim(a, i, jm2, k, w0);
        load_prim(a, i, jm1, k, w1);
        load_prim(a, i, jp1, k, w3);
        load_prim(a, i, jp2, k, w4);
        reconstruct<R, LIM>(w0, w1, wc, w3, wl, wr);
        face_flux<R, 2, FLUX>(wl, wr, a.gam, a.igm1, fm);
        reconstruct<R, LIM>(w1, wc, w3, w4, wl, wr);
        face_flux<R, 2, FLUX>(wl, wr, a.gam, a.igm1, fp);
        const R sm = a.m.sm[j], sp = a.m.sp[j], ict = a.m.ict[j];
#pragma unroll
        for (int v = 0; v < NV; ++v) L[v] -= hr * (sp * fp[v] - sm * fm[v]) * ict;
      }
      {  // phi faces, periodic
        R w0[NV], w1[NV], w3[NV], w4[NV], wl[NV], wr[NV], fm[NV], fp[NV];
        const int np = a.np;
        const int km2 = (k - 2 + 2 * np) % np, km1 = (k - 1 + np) % np;
        const int kp1 = (k + 1) % np, kp2 = (k + 2) % np;
        load_prim(a, i, j, km2, w0);
        load_prim(a, i, j, km1, w1);
        load_prim(a, i, j, kp1, w3);
        load_prim(a, i, j, kp2, w4);
        reconstruct<R, LIM>(w0, w1, wc, w3, wl, wr);
        face_flux<R, 3, FLUX>(wl, wr, a.gam, a.igm1, fm);
        reconstruct<R, LIM>(w1, wc, w3, w4, wl, wr);
        face_flux<R, 3, FLUX>(wl, wr, a.gam, a.igm1, fp);
        const R f = hr * a.m.phf[j];
#pragma unroll
        for (int v = 0; v < NV; ++v) L[v] -= f * (fp[v] - fm[v]);
      }
      add_sources<R>(wc, a.m, i, j, a.omega, a.gravity, a.corot, L);
      R uc[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) uc[v] = a.uin[v * a.ncell + c];
      if (STAGE == 1) {
#pragma unroll
        for (int v = 0; v < NV; ++v) a.uout[v * a.ncell + c] = uc[v] + dt * L[v];
      } else {
        R un[NV], unew[NV], wn[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          un[v] = a.un[v * a.ncell + c];
          unew[v] = R(0.5) * un[v] + R(0.5) * (uc[v] + dt * L[v]);
          a.uout[v * a.ncell + c] = unew[v];
        }
        cons2prim<R>(unew, wn, a.gm1);
        lam = cell_rate<R>(wn, a.m, i, j, a.gam);
        const double d = (double)unew[0] - (double)un[0];
        s1 = d * d;
        s0 = (double)un[0] * (double)un[0];
        if (!cell_valid<R>(unew, wn)) bad = (int)c;
      }
    }
  }
  if (STAGE == 2 && active)
    finish_reduction(a.clock, a.partials, gridDim.x * gridDim.y * gridDim.z, a.cfl, 1, lam, s1,
                     s0, bad);
}

// CFL dt of the current state; no time advance.
template <typename R>
__global__ void __launch_bounds__(256) k_cfl(StageArgs<R> a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int k = blockIdx.z;
  double lam = 0.0;
  int bad = BAD_NONE;
  if (i < a.nr && j < a.nt) {
    const long long c = ((long long)k * a.nt + j) * a.nr + i;
    R u[NV], w[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) u[v] = a.uin[v * a.ncell + c];
    cons2prim<R>(u, w, a.gm1);
    lam = cell_rate<R>(w, a.m, i, j, a.gam);
  }
  // invalid cells are reported by the next step, not here
  finish_reduction(a.clock, a.partials, gridDim.x * gridDim.y * gridDim.z, a.cfl, 0, lam, 0.0,
                   0.0, bad);
}

template <typename R, int FLUX, int LIM>
static void launch_stage_t(const StageArgs<R>& a, int stage, dim3 grid, dim3 blk, hipStream_t s) {
  if (stage == 1)
    hipLaunchKernelGGL((k_stage_v1<R, FLUX, LIM, 1>), grid, blk, 0, s, a);
  else
    hipLaunchKernelGGL((k_stage_v1<R, FLUX, LIM, 2>), grid, blk, 0, s, a);
}

template <typename R>
void launch_stage(const StageArgs<R>& a, int stage, int flux, int lim, dim3 grid, dim3 blk,
                  hipStream_t s) {
  if (flux == FLUX_TVDLF) {
    if (lim == LIM_MINMOD) launch_stage_t<R, FLUX_TVDLF, LIM_MINMOD>(a, stage, grid, blk, s);
    else launch_stage_t<R, FLUX_TVDLF, LIM_MC>(a, stage, grid, blk, s);
  } else {
    if (lim == LIM_MINMOD) launch_stage_t<R, FLUX_HLL, LIM_MINMOD>(a, stage, grid, blk, s);
    else launch_stage_t<R, FLUX_HLL, LIM_MC>(a, stage, grid, blk, s);
  }
}
template void launch_stage<double>(const StageArgs<double>&, int, int, int, dim3, dim3,
                                   hipStream_t);
template void launch_stage<float>(const StageArgs<float>&, int, int, int, dim3, dim3,
                                  hipStream_t);

template <typename R>
void launch_cfl(const StageArgs<R>& a, dim3 grid, dim3 blk, hipStream_t s) {
  hipLaunchKernelGGL(k_cfl<R>, grid, blk, 0, s, a);
}
template void launch_cfl<double>(const StageArgs<double>&, dim3, dim3, hipStream_t);
template void launch_cfl<float>(const StageArgs<float>&, dim3, dim3, hipStream_t);

// ------------------------------------------------- init and conversions --
// Radial expansion of map 0 from r_in (Sect. 2.1).
template <typename R>
__global__ void k_init_radial(BndArgs b, const double* __restrict__ m64, R* __restrict__ u,
                              int nr, double gam) {
  const long long n = (long long)nr * b.nt * b.np;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int i = (int)(c % nr);
  const int j = (int)((c / nr) % b.nt);
  const int k = (int)(c / ((long long)nr * b.nt));
  const long long plane = (long long)b.nt * b.np;
  const long long q = (long long)j * b.np + k;
  const double rc = m64[8 * nr + i];
  const double x = b.r_in / rc;
  const double sth = sin(b.tc[j]);
  double w[NV];
  w[0] = b.maps[0 * plane + q] * x * x;
  w[1] = b.maps[1 * plane + q];
  w[2] = 0.0;
  w[3] = -b.omega * rc * sth;
  w[4] = b.maps[4 * plane + q] * pow(x, 2.0 * gam);
  w[5] = b.maps[5 * plane + q] * x * x;
  w[6] = 0.0;
  w[7] = b.maps[7 * plane + q] * x;
  double uu[NV];
  prim2cons<double>(w, uu, 1.0 / (gam - 1.0));
  for (int v = 0; v < NV; ++v) u[v * n + c] = (R)uu[v];
}

template <typename R>
void launch_init_radial(const BndArgs& b, const double* m64, void* u, int nr, double gam,
                        hipStream_t s) {
  const long long n = (long long)nr * b.nt * b.np;
  hipLaunchKernelGGL(k_init_radial<R>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, b,
                     m64, (R*)u, nr, gam);
}
template void launch_init_radial<double>(const BndArgs&, const double*, void*, int, double,
                                         hipStream_t);
template void launch_init_radial<float>(const BndArgs&, const double*, void*, int, double,
                                        hipStream_t);

// kind 0: primitive SI <-> state; kind 1: conservative code units <-> state.
template <typename R>
__global__ void k_import(const double* __restrict__ in, R* __restrict__ u, long long n, int kind,
                         Scale sc, double gam) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  double a[NV], uu[NV];
  for (int v = 0; v < NV; ++v) a[v] = in[v * n + c];
  if (kind == 0) {
    for (int v = 0; v < NV; ++v) a[v] /= sc.s[v];
    prim2cons<double>(a, uu, 1.0 / (gam - 1.0));
  } else {
    for (int v = 0; v < NV; ++v) uu[v] = a[v];
  }
  for (int v = 0; v < NV; ++v) u[v * n + c] = (R)uu[v];
}

template <typename R>
__global__ void k_export(const R* __restrict__ u, double* __restrict__ out, long long n, int kind,
                         Scale sc, double gam) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  double uu[NV], w[NV];
  for (int v = 0; v < NV; ++v) uu[v] = (double)u[v * n + c];
  if (kind == 0) {
    cons2prim<double>(uu, w, gam - 1.0);
    for (int v = 0; v < NV; ++v) out[v * n + c] = w[v] * sc.s[v];
  } else {
    for (int v = 0; v < NV; ++v) out[v * n + c] = uu[v];
  }
}

template <typename R>
void launch_import(const double* in, void* u, long long n, int kind, const Scale& sc, double gam,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_import<R>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, (R*)u,
                     n, kind, sc, gam);
}
template <typename R>
void launch_export(const void* u, double* out, long long n, int kind, const Scale& sc, double gam,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_export<R>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     (const R*)u, out, n, kind, sc, gam);
}
template void launch_import<double>(const double*, void*, long long, int, const Scale&, double,
                                    hipStream_t);
template void launch_import<float>(const double*, void*, long long, int, const Scale&, double,
                                   hipStream_t);
template void launch_export<double>(const void*, double*, long long, int, const Scale&, double,
                                    hipStream_t);
template void launch_export<float>(const void*, double*, long long, int, const Scale&, double,
                                   hipStream_t);

// ---------------------------------------------------------------- probes --
// Position from the trajectory table at time t (clamped), co-rotating
// longitude phi - Omega t, trilinear interpolation of the primitives between
// the 8 surrounding cell centres (linear in r on the stretched grid,
// periodic in phi), v_phi returned in the inertial frame.
template <typename R>
__device__ void probe_eval(const ProbeArgs& a, const R* __restrict__ u, int q, double tcode,
                           double* o) {
  const double ts = tcode * a.sc.t;
  const double* tb = a.traj + (long long)q * a.npts * 4;
  double pos[4];
  const int np = a.npts;
  if (np == 1 || ts <= tb[0]) {
    for (int e = 0; e < 4; ++e) pos[e] = tb[e];
  } else if (ts >= tb[(np - 1) * 4]) {
    for (int e = 0; e < 4; ++e) pos[e] = tb[(np - 1) * 4 + e];
  } else {
    int lo = 0, hi = np - 1;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (tb[mid * 4] <= ts) lo = mid; else hi = mid;
    }
    const double al = (ts - tb[lo * 4]) / (tb[(lo + 1) * 4] - tb[lo * 4]);
    pos[0] = ts;
    for (int e = 1; e < 4; ++e) pos[e] = (1.0 - al) * tb[lo * 4 + e] + al * tb[(lo + 1) * 4 + e];
  }
  const double twopi = 6.283185307179586476925286766559;
  const double r = pos[1] / a.sc.len, th = pos[2];
  double ph = pos[3] - a.omega * tcode;
  ph = ph - floor(ph / twopi) * twopi;
  o[0] = ts;
  o[1] = pos[1];
  o[2] = th;
  o[3] = ph;
  const int nr = a.nr, nt = a.nt, nph = a.np;
  const double* rc = a.rc;
  const double* tc = a.tc;
  if (!(r >= rc[0] && r <= rc[nr - 1] && th >= tc[0] && th <= tc[nt - 1])) {
    for (int v = 0; v < NV; ++v) o[4 + v] = __builtin_nan("");
    return;
  }
  int lo = 0, hi = nr - 1;  // rc[lo] <= r, lo <= nr-2
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (rc[mid] <= r) lo = mid; else hi = mid;
  }
  const int i = lo;
  int jl = 0, jh = nt - 1;
  while (jh - jl > 1) {
    const int mid = (jl + jh) >> 1;
    if (tc[mid] <= th) jl = mid; else jh = mid;
  }
  const int j = jl;
  const double fk = (ph - 0.5 * a.dph) / a.dph;
  const int k0 = (int)floor(fk);
  const double az = fk - k0;
  const int ka = ((k0 % nph) + nph) % nph, kb = (ka + 1) % nph;
  const double ax = (r - rc[i]) / (rc[i + 1] - rc[i]);
  const double ay = (th - tc[j]) / (tc[j + 1] - tc[j]);
  const long long n = (long long)nr * nt * nph;
  double acc[NV] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int cz = 0; cz < 2; ++cz)
    for (int cy = 0; cy < 2; ++cy)
      for (int cx = 0; cx < 2; ++cx) {
        const double wt = (cx ? ax : 1.0 - ax) * (cy ? ay : 1.0 - ay) * (cz ? az : 1.0 - az);
        const long long c = ((long long)(cz ? kb : ka) * nt + (j + cy)) * nr + (i + cx);
        double uu[NV], w[NV];
        for (int v = 0; v < NV; ++v) uu[v] = (double)u[v * n + c];
        cons2prim<double>(uu, w, a.gam - 1.0);
        for (int v = 0; v < NV; ++v) acc[v] += wt * w[v];
      }
  acc[3] += a.omega * r * sin(th);
  for (int v = 0; v < NV; ++v) o[4 + v] = acc[v] * a.sc.s[v];
}

template <typename R>
__global__ void k_probe_sample(ProbeArgs a, const DevClock* __restrict__ ck,
                               const R* __restrict__ u, double* __restrict__ out) {
  const int q = threadIdx.x;
  if (q < a.n) probe_eval<R>(a, u, q, ck->t, out + 12 * q);
}

// Append a record after a completed step when the cadence rule fires.
template <typename R>
__global__ void k_probe_log(ProbeArgs a, DevClock* ck, const R* __restrict__ u,
                            double* __restrict__ log) {
  const int q = threadIdx.x;
  const int adv = ck->advanced;
  const double t = ck->t;
  long long idx = 0;
  bool rec = adv != 0;
  if (rec && a.cadence > 0.0) {
    idx = (long long)floor(t * a.sc.t / a.cadence);
    rec = idx > ck->last_sample;
  }
  const long long row = ck->n_log;
  __syncthreads();
  if (rec && row < a.log_rows && q < a.n)
    probe_eval<R>(a, u, q, t, log + (row * a.max_probes + q) * 12);
  __syncthreads();
  if (q == 0) {
    if (rec) {
      ck->n_log = row + 1;
      if (a.cadence > 0.0) ck->last_sample = idx;
    }
    ck->advanced = 0;
  }
}

template <typename R>
void launch_probe_sample(const ProbeArgs& a, const DevClock* ck, const void* u, double* out,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_probe_sample<R>, dim3(1), dim3(64), 0, s, a, ck, (const R*)u, out);
}
template <typename R>
void launch_probe_log(const ProbeArgs& a, DevClock* ck, const void* u, double* log,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_probe_log<R>, dim3(1), dim3(64), 0, s, a, ck, (const R*)u, log);
}
template void launch_probe_sample<double>(const ProbeArgs&, const DevClock*, const void*, double*,
                                          hipStream_t);
template void launch_probe_sample<float>(const ProbeArgs&, const DevClock*, const void*, double*,
                                         hipStream_t);
template void launch_probe_log<double>(const ProbeArgs&, DevClock*, const void*, double*,
                                       hipStream_t);
template void launch_probe_log<float>(const ProbeArgs&, DevClock*, const void*, double*,
                                      hipStream_t);

}  // namespace icr
