// icr_kernels.hip -- HIP kernels of the heliospheric MHD hot path (gfx950).
//
//   k_metric        per-r / per-theta metric factors of the stretched
//                   spherical grid (radially stretched grid, Sect. 2)
//   k_boundary      inner-boundary primitives at the two RK stage times:
//                   time interpolation between maps (Sect. 3) and the
//                   cone-CME overwrite (Sect. 3.2); one value serves both
//                   ghost layers (Sect. 2.1)
//   k_stage_v1      fused reconstruct + flux + divergence + sources + RK2
//                   combine (Sect. 2 Eqs. 1-6), one thread per cell, every
//                   neighbour converted on the fly (reference variant; the
//                   default face-once variant is in icr_stage_lds.hip);
//                   stage 2 also writes per-block CFL / residual partials
//   k_cfl           CFL partials of the current state (after init / set_state)
//   k_probe_sample  trajectory interpolation, frame change and trilinear
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
template <typename R>
__global__ void k_boundary(BndArgs a, const DevClock* __restrict__ ck, R* __restrict__ g1,
                           R* __restrict__ g2, R* __restrict__ tg1, R* __restrict__ tg2) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int plane = a.nt * a.np;
  if (q >= plane || !ck->active) return;
  const int j = q % a.nt, k = q / a.nt;
  double w[NV];
  int in1, in2;
  boundary_prim(a, ck->t, j, k, w, &in1);
  for (int v = 0; v < NV; ++v) g1[(long long)v * plane + q] = (R)w[v];
  boundary_prim(a, ck->t + ck->dt, j, k, w, &in2);
  for (int v = 0; v < NV; ++v) g2[(long long)v * plane + q] = (R)w[v];
  // tracer of the inner ghost cells: CME material inside an inserted cone
  if (tg1) {
    tg1[q] = (R)in1;
    tg2[q] = (R)in2;
  }
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

void launch_boundary(const BndArgs& a, const DevClock* ck, void* g1, void* g2, void* tg1,
                     void* tg2, bool f32, hipStream_t s) {
  const int plane = a.nt * a.np;
  const dim3 grid((plane + 255) / 256), blk(256);
  if (f32)
    hipLaunchKernelGGL(k_boundary<float>, grid, blk, 0, s, a, ck, (float*)g1, (float*)g2,
                       (float*)tg1, (float*)tg2);
  else
    hipLaunchKernelGGL(k_boundary<double>, grid, blk, 0, s, a, ck, (double*)g1, (double*)g2,
                       (double*)tg1, (double*)tg2);
}

void launch_boundary_at(const BndArgs& a, double t, double* out, const Scale& sc, hipStream_t s) {
  const int plane = a.nt * a.np;
  hipLaunchKernelGGL(k_boundary_at, dim3((plane + 255) / 256), dim3(256), 0, s, a, t, out, sc);
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
    if (a.asymm) {  // transverse parts: minus the mirror cell -1 - i
      const long long c = ((long long)k * a.nt + j) * a.nr + (-1 - i);
      R u[NV], wm[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) u[v] = a.uin[v * a.ncell + c];
      cons2prim<R>(u, wm, a.gm1);
      w[2] = -wm[2];
      w[3] = -wm[3];
      w[6] = -wm[6];
      w[7] = -wm[7];
    }
    return;
  }
  if (i >= a.nr) i = a.nr - 1;
  const long long c = ((long long)k * a.nt + j) * a.nr + i;
  R u[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = a.uin[v * a.ncell + c];
  cons2prim<R>(u, w, a.gm1);
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
        if constexpr (LIM == LIM_WENO5) {
          R wm3[NV], wp3[NV];
          load_prim(a, i - 3, j, k, wm3);
          load_prim(a, i + 3, j, k, wp3);
          reconstruct_weno5<R>(wm3, w0, w1, wc, w3, w4, wl, wr);
          face_flux<R, 1, FLUX>(wl, wr, a.gam, a.igm1, fm);
          reconstruct_weno5<R>(w0, w1, wc, w3, w4, wp3, wl, wr);
          face_flux<R, 1, FLUX>(wl, wr, a.gam, a.igm1, fp);
        } else {
          reconstruct<R, LIM>(w0, w1, wc, w3, wl, wr);
          face_flux<R, 1, FLUX>(wl, wr, a.gam, a.igm1, fm);
          reconstruct<R, LIM>(w1, wc, w3, w4, wl, wr);
          face_flux<R, 1, FLUX>(wl, wr, a.gam, a.igm1, fp);
        }
        const R rm2 = a.m.rm2[i], rp2 = a.m.rp2[i], ivr = a.m.ivr[i];
#pragma unroll
        for (int v = 0; v < NV; ++v) L[v] -= (rp2 * fp[v] - rm2 * fm[v]) * ivr;
        if (a.fmass) {
          a.fmass[c] = fm[0];
          if (i == a.nr - 1) a.fmass_rout[(long long)k * a.nt + j] = fp[0];
        }
      }
      const R hr = a.m.hr[i];
      {  // theta faces, mirror rows beyond the (reflecting) colatitude edges
        R w0[NV], w1[NV], w3[NV], w4[NV], wl[NV], wr[NV], fm[NV], fp[NV];
        bool f0, f1, f3, f4;
        const int jm2 = mirror_row(j - 2, a.nt, f0), jm1 = mirror_row(j - 1, a.nt, f1);
        const int jp1 = mirror_row(j + 1, a.nt, f3), jp2 = mirror_row(j + 2, a.nt, f4);
        load_prim(a, i, jm2, k, w0);
        load_prim(a, i, jm1, k, w1);
        load_prim(a, i, jp1, k, w3);
        load_prim(a, i, jp2, k, w4);
        if (f0) flip_theta(w0);
        if (f1) flip_theta(w1);
        if (f3) flip_theta(w3);
        if (f4) flip_theta(w4);
        if constexpr (LIM == LIM_WENO5) {
          R wm3[NV], wp3[NV];
          bool fm3, fp3;
          load_prim(a, i, mirror_row(j - 3, a.nt, fm3), k, wm3);
          load_prim(a, i, mirror_row(j + 3, a.nt, fp3), k, wp3);
          if (fm3) flip_theta(wm3);
          if (fp3) flip_theta(wp3);
          reconstruct_weno5<R>(wm3, w0, w1, wc, w3, w4, wl, wr);
          face_flux<R, 2, FLUX>(wl, wr, a.gam, a.igm1, fm);
          reconstruct_weno5<R>(w0, w1, wc, w3, w4, wp3, wl, wr);
          face_flux<R, 2, FLUX>(wl, wr, a.gam, a.igm1, fp);
        } else {
          reconstruct<R, LIM>(w0, w1, wc, w3, wl, wr);
          face_flux<R, 2, FLUX>(wl, wr, a.gam, a.igm1, fm);
          reconstruct<R, LIM>(w1, wc, w3, w4, wl, wr);
          face_flux<R, 2, FLUX>(wl, wr, a.gam, a.igm1, fp);
        }
        const R sm = a.m.sm[j], sp = a.m.sp[j], ict = a.m.ict[j];
#pragma unroll
        for (int v = 0; v < NV; ++v) L[v] -= hr * (sp * fp[v] - sm * fm[v]) * ict;
        if (a.fmass) {
          a.fmass[a.ncell + c] = fm[0];
          if (j == a.nt - 1) a.fmass_tend[(long long)k * a.nr + i] = fp[0];
        }
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
        if constexpr (LIM == LIM_WENO5) {
          R wm3[NV], wp3[NV];
          load_prim(a, i, j, ((k - 3) % np + np) % np, wm3);
          load_prim(a, i, j, (k + 3) % np, wp3);
          reconstruct_weno5<R>(wm3, w0, w1, wc, w3, w4, wl, wr);
          face_flux<R, 3, FLUX>(wl, wr, a.gam, a.igm1, fm);
          reconstruct_weno5<R>(w0, w1, wc, w3, w4, wp3, wl, wr);
          face_flux<R, 3, FLUX>(wl, wr, a.gam, a.igm1, fp);
        } else {
          reconstruct<R, LIM>(w0, w1, wc, w3, wl, wr);
          face_flux<R, 3, FLUX>(wl, wr, a.gam, a.igm1, fm);
          reconstruct<R, LIM>(w1, wc, w3, w4, wl, wr);
          face_flux<R, 3, FLUX>(wl, wr, a.gam, a.igm1, fp);
        }
        const R f = hr * a.m.phf[j];
#pragma unroll
        for (int v = 0; v < NV; ++v) L[v] -= f * (fp[v] - fm[v]);
        if (a.fmass) a.fmass[2 * a.ncell + c] = fm[0];
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
    write_partials(a.partials, (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x,
                   lam, s1, s0, bad);
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
  write_partials(a.partials, (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x,
                 lam, 0.0, 0.0, bad);
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
    else if (lim == LIM_WENO5) launch_stage_t<R, FLUX_TVDLF, LIM_WENO5>(a, stage, grid, blk, s);
    else launch_stage_t<R, FLUX_TVDLF, LIM_MC>(a, stage, grid, blk, s);
  } else if (flux == FLUX_HLLD) {
    if (lim == LIM_MINMOD) launch_stage_t<R, FLUX_HLLD, LIM_MINMOD>(a, stage, grid, blk, s);
    else if (lim == LIM_WENO5) launch_stage_t<R, FLUX_HLLD, LIM_WENO5>(a, stage, grid, blk, s);
    else launch_stage_t<R, FLUX_HLLD, LIM_MC>(a, stage, grid, blk, s);
  } else {
    if (lim == LIM_MINMOD) launch_stage_t<R, FLUX_HLL, LIM_MINMOD>(a, stage, grid, blk, s);
    else if (lim == LIM_WENO5) launch_stage_t<R, FLUX_HLL, LIM_WENO5>(a, stage, grid, blk, s);
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
// Cells c0 .. c0+m-1 of the state (variable stride ncell); the buffer holds
// those m cells with variable stride ld (ld = ncell, c0 = 0 for a whole
// state in place, ld = m for a staging chunk).
template <typename R>
__global__ void k_import(const double* __restrict__ in, long long ld, R* __restrict__ u,
                         long long ncell, long long c0, long long m, int kind, Scale sc,
                         double gam) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m) return;
  double a[NV], uu[NV];
  for (int v = 0; v < NV; ++v) a[v] = in[v * ld + c];
  if (kind == 0) {
    for (int v = 0; v < NV; ++v) a[v] /= sc.s[v];
    prim2cons<double>(a, uu, 1.0 / (gam - 1.0));
  } else {
    for (int v = 0; v < NV; ++v) uu[v] = a[v];
  }
  for (int v = 0; v < NV; ++v) u[v * ncell + c0 + c] = (R)uu[v];
}

template <typename R>
__global__ void k_export(const R* __restrict__ u, long long ncell, long long c0, long long m,
                         double* __restrict__ out, long long ld, int kind, Scale sc, double gam) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m) return;
  double uu[NV], w[NV];
  for (int v = 0; v < NV; ++v) uu[v] = (double)u[v * ncell + c0 + c];
  if (kind == 0) {
    cons2prim<double>(uu, w, gam - 1.0);
    for (int v = 0; v < NV; ++v) out[v * ld + c] = w[v] * sc.s[v];
  } else {
    for (int v = 0; v < NV; ++v) out[v * ld + c] = uu[v];
  }
}

template <typename R>
void launch_import(const double* in, long long ld, void* u, long long ncell, long long c0,
                   long long m, int kind, const Scale& sc, double gam, hipStream_t s) {
  hipLaunchKernelGGL(k_import<R>, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, in, ld,
                     (R*)u, ncell, c0, m, kind, sc, gam);
}
template <typename R>
void launch_export(const void* u, long long ncell, long long c0, long long m, double* out,
                   long long ld, int kind, const Scale& sc, double gam, hipStream_t s) {
  hipLaunchKernelGGL(k_export<R>, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s,
                     (const R*)u, ncell, c0, m, out, ld, kind, sc, gam);
}
template void launch_import<double>(const double*, long long, void*, long long, long long,
                                    long long, int, const Scale&, double, hipStream_t);
template void launch_import<float>(const double*, long long, void*, long long, long long,
                                   long long, int, const Scale&, double, hipStream_t);
template void launch_export<double>(const void*, long long, long long, long long, double*,
                                    long long, int, const Scale&, double, hipStream_t);
template void launch_export<float>(const void*, long long, long long, long long, double*,
                                   long long, int, const Scale&, double, hipStream_t);

// ---------------------------------------------------------------- probes --
// Primitive rho and v_r on the sphere r (code units) for every (theta, phi)
// column, linear in r between the two bracketing cell centres (clamped to the
// first / last centre): out [2][nt][np], SI.
template <typename R>
__global__ void k_shell(const R* __restrict__ u, const double* __restrict__ rc, int nr, int nt,
                        int np, double r, double gam, Scale sc, double* __restrict__ out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nt * np) return;
  const int j = q / np, k = q % np;
  int i = 0;
  double a = 0.0;
  if (nr > 1 && r > rc[0]) {
    if (r >= rc[nr - 1]) {
      i = nr - 2;
      a = 1.0;
    } else {
      int lo = 0, hi = nr - 1;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (rc[mid] <= r) lo = mid; else hi = mid;
      }
      i = lo;
      a = (r - rc[i]) / (rc[i + 1] - rc[i]);
    }
  }
  const long long n = (long long)nr * nt * np;
  double res[2] = {0.0, 0.0};
  for (int c = 0; c < (nr > 1 ? 2 : 1); ++c) {
    const long long cell = ((long long)k * nt + j) * nr + i + c;
    double uu[NV], w[NV];
    for (int v = 0; v < NV; ++v) uu[v] = (double)u[v * n + cell];
    cons2prim<double>(uu, w, gam - 1.0);
    const double wt = c ? a : 1.0 - a;
    res[0] += wt * w[0];
    res[1] += wt * w[1];
  }
  out[q] = res[0] * sc.s[0];
  out[nt * np + q] = res[1] * sc.s[1];
}

template <typename R>
void launch_shell(const void* u, const double* rc, int nr, int nt, int np, double r, double gam,
                  const Scale& sc, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_shell<R>, dim3((nt * np + 255) / 256), dim3(256), 0, s, (const R*)u, rc,
                     nr, nt, np, r, gam, sc, out);
}
template void launch_shell<double>(const void*, const double*, int, int, int, double, double,
                                   const Scale&, double*, hipStream_t);
template void launch_shell<float>(const void*, const double*, int, int, int, double, double,
                                  const Scale&, double*, hipStream_t);

// ---------------------------------------------------- passive tracer --
// rho tau of every cell, one RK stage: the face flux is the stage's mass flux
// times tau = (rho tau) / rho of the upwind cell (the inner ghost carries 1
// inside an inserted CME cone, 0 elsewhere; beyond r_out and the colatitude
// edges the edge cell's own tau; periodic in phi), divergence with the same
// metric factors as the stage kernels, then the stage's RK combine.
template <typename R, int STAGE>
__global__ void __launch_bounds__(256) k_tracer(TracerArgs<R> a) {
  const long long c =
      (long long)xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  tracer_cell<R, STAGE>(a, c);
}

template <typename R>
void launch_tracer(const TracerArgs<R>& a, int stage, hipStream_t s) {
  const dim3 grid((unsigned)((a.ncell + 255) / 256)), blk(256);
  if (stage == 1)
    hipLaunchKernelGGL((k_tracer<R, 1>), grid, blk, 0, s, a);
  else
    hipLaunchKernelGGL((k_tracer<R, 2>), grid, blk, 0, s, a);
}
template void launch_tracer<double>(const TracerArgs<double>&, int, hipStream_t);
template void launch_tracer<float>(const TracerArgs<float>&, int, hipStream_t);

// cells c0 .. c0+m-1; tau holds those m cells
template <typename R>
__global__ void k_tracer_io(const R* __restrict__ u, R* __restrict__ t, double* __restrict__ tau,
                            long long c0, long long m, int to_state) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m) return;
  if (to_state)
    t[c0 + c] = u[c0 + c] * (R)tau[c];
  else
    tau[c] = (double)(t[c0 + c] / u[c0 + c]);
}

template <typename R>
void launch_tracer_io(const void* u, void* t, double* tau, long long c0, long long m,
                      int to_state, hipStream_t s) {
  hipLaunchKernelGGL(k_tracer_io<R>, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s,
                     (const R*)u, (R*)t, tau, c0, m, to_state);
}
template void launch_tracer_io<double>(const void*, void*, double*, long long, long long, int,
                                       hipStream_t);
template void launch_tracer_io<float>(const void*, void*, double*, long long, long long, int,
                                      hipStream_t);

// ------------------------------------------------- velocity divergence --
// Finite-volume divergence of the co-rotating-frame velocity with face
// velocities the mean of the two neighbouring cell centres (inner ghost from
// the boundary primitives, zero-gradient beyond r_out, mirror rows with
// v_theta negated beyond the colatitude edges, periodic phi), in 1/s.
template <typename R>
__global__ void __launch_bounds__(256) k_divv(StageArgs<R> a, BndArgs b, double inv_time,
                                              long long c0, long long m, double* out) {
  const long long q =
      (long long)xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (q >= m) return;
  const long long c = c0 + q;
  const int nr = a.nr, nt = a.nt, np = a.np;
  const int i = (int)(c % nr);
  const long long col = c / nr;
  const int j = (int)(col % nt), k = (int)(col / nt);
  R w0[NV], wm[NV], wp[NV];
  load_prim(a, i, j, k, w0);
  if (i > 0) {
    load_prim(a, i - 1, j, k, wm);
  } else {  // inner ghost: the boundary primitives at the current time
    double wb[NV];
    boundary_prim(b, a.clock->t, j, k, wb);
#pragma unroll
    for (int v = 0; v < NV; ++v) wm[v] = (R)wb[v];
  }
  load_prim(a, i + 1, j, k, wp);
  const R vr0 = R(0.5) * (wm[1] + w0[1]), vr1 = R(0.5) * (w0[1] + wp[1]);
  bool fm, fp;
  load_prim(a, i, mirror_row(j - 1, nt, fm), k, wm);
  load_prim(a, i, mirror_row(j + 1, nt, fp), k, wp);
  if (fm) flip_theta(wm);
  if (fp) flip_theta(wp);
  const R vt0 = R(0.5) * (wm[2] + w0[2]), vt1 = R(0.5) * (w0[2] + wp[2]);
  load_prim(a, i, j, (k + np - 1) % np, wm);
  load_prim(a, i, j, (k + 1) % np, wp);
  const R vp0 = R(0.5) * (wm[3] + w0[3]), vp1 = R(0.5) * (w0[3] + wp[3]);
  const R hr = a.m.hr[i];
  const R d = (a.m.rp2[i] * vr1 - a.m.rm2[i] * vr0) * a.m.ivr[i] +
              hr * (a.m.sp[j] * vt1 - a.m.sm[j] * vt0) * a.m.ict[j] +
              hr * a.m.phf[j] * (vp1 - vp0);
  out[q] = (double)d * inv_time;
}

template <typename R>
void launch_divv(const StageArgs<R>& a, const BndArgs& b, double inv_time_unit, long long c0,
                 long long m, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_divv<R>, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, a, b,
                     inv_time_unit, c0, m, out);
}
template void launch_divv<double>(const StageArgs<double>&, const BndArgs&, double, long long,
                                  long long, double*, hipStream_t);
template void launch_divv<float>(const StageArgs<float>&, const BndArgs&, double, long long,
                                 long long, double*, hipStream_t);

template <typename R>
__global__ void k_probe_sample(ProbeArgs a, const DevClock* __restrict__ ck,
                               const R* __restrict__ u, double* __restrict__ out) {
  const int q = threadIdx.x;
  if (q < a.n) probe_eval<R>(a, u, q, ck->t, out + 12 * q);
}

template <typename R>
void launch_probe_sample(const ProbeArgs& a, const DevClock* ck, const void* u, double* out,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_probe_sample<R>, dim3(1), dim3(64), 0, s, a, ck, (const R*)u, out);
}
template void launch_probe_sample<double>(const ProbeArgs&, const DevClock*, const void*, double*,
                                          hipStream_t);
template void launch_probe_sample<float>(const ProbeArgs&, const DevClock*, const void*, double*,
                                         hipStream_t);


// ------------------------------------------------ accuracy diagnostics --
// The FP64 reciprocal and square root of the face-once stage kernels
// (rcp_fast, sqrt_fast) on arbitrary inputs.
__global__ void k_fast_math(const double* __restrict__ x, long long n, double* __restrict__ rcp,
                            double* __restrict__ sq) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const double v = x[q];
  rcp[q] = rcp_fast(v);
  sq[q] = sqrt_fast(v);
}

void launch_fast_math(const double* x, long long n, double* rcp, double* sq, hipStream_t s) {
  hipLaunchKernelGGL(k_fast_math, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n, rcp,
                     sq);
}

}  // namespace icr
