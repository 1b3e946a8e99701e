// icr_kernels.hpp -- argument blocks and launchers shared by the kernel and
// host translation units of the HIP library.
#pragma once
#include <hip/hip_runtime.h>

#include "icr_device.hpp"

namespace icr {

// Metric arrays: R_ARRAYS per-r arrays of n_r, then T_ARRAYS per-theta
// arrays of n_theta, in the solver precision and in float64.  The float64
// block additionally holds the n_r+1 radial edges and the n_theta
// colatitude centres.
constexpr int R_ARRAYS = 9;  // r-^2, r+^2, 1/V_r, H_r, G_r, 1/r_c, -GM/r_c^2, 1/dr, r_c
constexpr int T_ARRAYS = 8;  // sin t-, sin t+, 1/C_t, cot, sin t_c, cos t_c, dt/(C_t dp), 1/(sin t_c dp)
inline __host__ __device__ long long OFF_REDGE64(int nr, int nt) {
  return (long long)R_ARRAYS * nr + (long long)T_ARRAYS * nt;
}
inline __host__ __device__ long long OFF_TC64(int nr, int nt) {
  return OFF_REDGE64(nr, nt) + nr + 1;
}
inline long long METRIC64_LEN(int nr, int nt) { return OFF_TC64(nr, nt) + nt; }
inline long long METRICR_LEN(int nr, int nt) {
  return (long long)R_ARRAYS * nr + (long long)T_ARRAYS * nt;
}

struct Scale {
  double s[NV];  // SI per code unit of each primitive channel
  double t;      // seconds per code time unit
  double len;    // metres per code length unit
};

struct MetricArgs {
  int nr, nt;
  double r_in, r_out, q;     // code units, q = (r_out/r_in)^(1/nr)
  double th_min, th_max;     // rad
  double dph;                // 2 pi / n_phi
  double gm;                 // GM in code units (0: no gravity)
  double* m64;
};

struct BndArgs {
  int nt, np;
  int n_maps;
  const double* tau;   // [n_maps] code time
  const double* maps;  // [n_maps][8][nt][np] code primitive
  int n_cme;
  const double* cme;   // [n][8]: t0, dur, colat, lon, cos(hw), v, rho, p (code)
  const double* tc;    // [nt] colatitude centres
  double dph, omega, r_in;
};

template <typename R>
struct StageArgs {
  const R* __restrict__ uin;   // state L acts on
  const R* __restrict__ un;    // U^n (stage-2 combine)
  R* __restrict__ uout;
  const R* __restrict__ ghost; // inner-boundary primitives [8][np][nt]
  Metric<R> m;
  DevClock* clock;
  double* partials;            // [blocks][4]
  int nr, nt, np;
  long long ncell;
  R gam, gm1, igm1, omega;
  double cfl;
  int gravity, corot;
  // 1: v_theta, v_phi, B_theta, B_phi of inner ghost layer g are minus those
  // of active cell g-1 (the paper's asymm rule); 0: the ghost primitives
  int asymm;
  // optional (passive tracer on): face mass fluxes of this stage, the lower
  // r / theta / phi face of every cell [3][ncell], the outer r face [np][nt]
  // and the upper theta face of the last row [np][nr]
  R* __restrict__ fmass;
  R* __restrict__ fmass_rout;
  R* __restrict__ fmass_tend;
};

// Passive tracer stage: rho tau advected with the stage's mass fluxes.
template <typename R>
struct TracerArgs {
  const R* __restrict__ tin;   // rho tau the stage starts from
  const R* __restrict__ tn;    // rho tau at t^n (stage-2 combine)
  R* __restrict__ tout;
  const R* __restrict__ rho;   // density the stage starts from (stride 1)
  const R* __restrict__ fm;    // [3][ncell] lower-face mass fluxes
  const R* __restrict__ frout; // [np][nt]
  const R* __restrict__ ftend; // [np][nr]
  const R* __restrict__ gtau;  // [np][nt] tau of the inner ghost cells
  Metric<R> m;
  const DevClock* clock;
  int nr, nt, np;
  long long ncell;
};

// One cell of a passive-tracer stage: upwind rho tau fluxes from the stage's
// face mass fluxes, then the stage update (stage 2: the RK2 combine with tn).
template <typename R, int STAGE>
__device__ __forceinline__ void tracer_cell(const TracerArgs<R>& a, long long c) {
  if (c >= a.ncell) return;
  const int nr = a.nr, nt = a.nt, np = a.np;
  const int i = (int)(c % nr);
  const long long col = c / nr;
  const int j = (int)(col % nt), k = (int)(col / nt);
  if (!a.clock->active) {
    if (STAGE == 2) a.tout[c] = a.tn[c];
    return;
  }
  const long long n = a.ncell, pc = (long long)nt * nr;
  auto tau = [&](long long q) { return a.tin[q] / a.rho[q]; };
  const R tc = tau(c);
  // r faces i-1/2, i+1/2
  const R fr0 = a.fm[c];
  const R fr1 = i + 1 < nr ? a.fm[c + 1] : a.frout[(long long)k * nt + j];
  const R tr0 = i > 0 ? tau(c - 1) : a.gtau[(long long)k * nt + j];
  const R tr1 = i + 1 < nr ? tau(c + 1) : tc;
  const R gr0 = fr0 * (fr0 >= R(0) ? tr0 : tc), gr1 = fr1 * (fr1 >= R(0) ? tc : tr1);
  // theta faces j-1/2, j+1/2
  const R ft0 = a.fm[n + c];
  const R ft1 = j + 1 < nt ? a.fm[n + c + nr] : a.ftend[(long long)k * nr + i];
  const R tt0 = j > 0 ? tau(c - nr) : tc;
  const R tt1 = j + 1 < nt ? tau(c + nr) : tc;
  const R gt0 = ft0 * (ft0 >= R(0) ? tt0 : tc), gt1 = ft1 * (ft1 >= R(0) ? tc : tt1);
  // phi faces k-1/2, k+1/2 (periodic)
  const long long cm = c + (k > 0 ? -pc : (long long)(np - 1) * pc);
  const long long cp = c + (k + 1 < np ? pc : -(long long)(np - 1) * pc);
  const R fp0 = a.fm[2 * n + c], fp1 = a.fm[2 * n + cp];
  const R gp0 = fp0 * (fp0 >= R(0) ? tau(cm) : tc), gp1 = fp1 * (fp1 >= R(0) ? tc : tau(cp));
  const R hr = a.m.hr[i];
  R L = R(0);
  L -= (a.m.rp2[i] * gr1 - a.m.rm2[i] * gr0) * a.m.ivr[i];
  L -= hr * (a.m.sp[j] * gt1 - a.m.sm[j] * gt0) * a.m.ict[j];
  L -= hr * a.m.phf[j] * (gp1 - gp0);
  const R dt = (R)a.clock->dt;
  if (STAGE == 1)
    a.tout[c] = a.tin[c] + dt * L;
  else
    a.tout[c] = R(0.5) * a.tn[c] + R(0.5) * (a.tin[c] + dt * L);
}

struct ProbeArgs {
  int n, npts, max_probes;
  long long log_rows;
  const double* traj;  // [n][npts][4] SI
  double cadence;      // s
  Scale sc;
  double omega, gam;   // code
  int nr, nt, np;
  const double* rc;    // [nr] code
  const double* tc;    // [nt]
  double dph;
};


// ------------------------------------------------------ shared helpers --
constexpr int NXCD = 8;  // accelerator complex dies of MI355X

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2): remap workgroup b of nb so that XCD x gets a contiguous range of
// tiles / cells, and neighbours that share data run on the same L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int xcd = b % NXCD, per = nb / NXCD, rem = nb % NXCD;
  return xcd * per + (xcd < rem ? xcd : rem) + b / NXCD;
}

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

__device__ inline void set_next_dt(DevClock* ck, double dtc) {
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

// Plain store of one block's partials; the finalize kernel reads them after
// the kernel boundary.
__device__ __forceinline__ void write_partials(double* partials, int bid, double lam, double s1,
                                               double s0, int bad) {
  __shared__ double sh[4][4];
  block_reduce(lam, s1, s0, bad, sh);
  if (threadIdx.x == 0 && threadIdx.y == 0) {
    partials[4 * bid + 0] = lam;
    partials[4 * bid + 1] = s1;
    partials[4 * bid + 2] = s0;
    partials[4 * bid + 3] = (double)bad;
  }
}

// CFL rate of one cell from its primitives: sum_d (|v_d| + c_f,d) / dx_d.
template <typename R, bool FAST = false, typename CM>
__device__ __forceinline__ double cell_rate_cm(const R (&w)[NV], const CM& cm, R gam) {
  const R lr = (fabs(w[1]) + cfast<R, 1, FAST>(w, gam)) * cm.r(MR_IDR);
  const R lt = (fabs(w[2]) + cfast<R, 2, FAST>(w, gam)) * cm.r(MR_IRC) * cm.ilth();
  const R lp = (fabs(w[3]) + cfast<R, 3, FAST>(w, gam)) * cm.r(MR_IRC) * cm.t(MT_ILPH);
  return (double)(lr + lt + lp);
}
template <typename R, bool FAST = false>
__device__ __forceinline__ double cell_rate(const R (&w)[NV], const Metric<R>& m, int i, int j,
                                            R gam) {
  return cell_rate_cm<R, FAST>(w, CellMetric<R>{m, i, j}, gam);
}

template <typename R>
__device__ __forceinline__ bool cell_valid(const R (&u)[NV], const R (&w)[NV]) {
  bool ok = w[0] > R(0) && w[4] > R(0);
#pragma unroll
  for (int v = 0; v < NV; ++v) ok = ok && isfinite(u[v]);
  return ok;
}

// Position from the trajectory table at time t (clamped), co-rotating
// longitude phi - Omega t, trilinear interpolation of the primitives between
// the 8 surrounding cell centres (linear in r on the stretched grid,
// periodic in phi), v_phi returned in the inertial frame.
template <typename R>
__device__ inline void probe_eval(const ProbeArgs& a, const R* __restrict__ u, int q, double tcode,
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

// Primitive at the inner shell for column (j, k) at code time t; *inside
// (optional) is set to 1 when a cone CME is being inserted there.
__device__ inline void boundary_prim(const BndArgs& a, double t, int j, int k, double (&w)[NV],
                                     int* inside = nullptr) {
  if (inside) *inside = 0;
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
        if (inside) *inside = 1;
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
Metric<R> metric_view(const R* base, int nr, int nt, double dth);

void launch_metric(const MetricArgs& a, void* mr, bool f32, hipStream_t s);
void launch_boundary(const BndArgs& a, const DevClock* ck, void* g1, void* g2, void* tg1,
                     void* tg2, bool f32,
                     hipStream_t s);
void launch_boundary_at(const BndArgs& a, double t, double* out, const Scale& sc, hipStream_t s);
void launch_clock_begin(DevClock* ck, double t_end, hipStream_t s);
template <typename R>
void launch_stage(const StageArgs<R>& a, int stage, int flux, int lim, dim3 grid, dim3 blk,
                  hipStream_t s);
template <typename R>
void launch_cfl(const StageArgs<R>& a, dim3 grid, dim3 blk, hipStream_t s);
template <typename R>
void launch_init_radial(const BndArgs& b, const double* m64, void* u, int nr, double gam,
                        hipStream_t s);
// cells c0 .. c0+m-1 of a state with ncell cells; the double buffer holds
// them with variable stride ld
template <typename R>
void launch_import(const double* in, long long ld, void* u, long long ncell, long long c0,
                   long long m, int kind, const Scale& sc, double gam, hipStream_t s);
template <typename R>
void launch_export(const void* u, long long ncell, long long c0, long long m, double* out,
                   long long ld, int kind, const Scale& sc, double gam, hipStream_t s);
template <typename R>
void launch_probe_sample(const ProbeArgs& a, const DevClock* ck, const void* u, double* out,
                         hipStream_t s);
template <typename R>
void launch_tracer(const TracerArgs<R>& a, int stage, hipStream_t s);
// tau [np][nt][nr] (host layout, device memory) <-> rho tau, with rho the
// density of state u
template <typename R>
void launch_tracer_io(const void* u, void* t, double* tau, long long c0, long long m,
                      int to_state, hipStream_t s);
// velocity divergence [1/s] of cells c0 .. c0+m-1 of state a.uin into
// out[0 .. m); inner ghost from the boundary maps / CMEs at the clock's time
template <typename R>
void launch_divv(const StageArgs<R>& a, const BndArgs& b, double inv_time_unit, long long c0,
                 long long m, double* out, hipStream_t s);
template <typename R>
void launch_shell(const void* u, const double* rc, int nr, int nt, int np, double r, double gam,
                  const Scale& sc, double* out, hipStream_t s);
template <typename R>
void launch_stage_lds(const StageArgs<R>& a, int stage, int flux, int lim, int tile_r,
                      int kplanes, hipStream_t s);
// Cells along r updated by a face-once tile of tile_r lanes: two lanes on
// each side carry the r halo.
__host__ __device__ constexpr int tile_cells_r(int tile_r) { return tile_r - 4; }
long long stage_lds_blocks(int nr, int nt, int np, int tile_r, int kplanes);
// the WENO5 face-once tile (64 x 4 threads, three-cell halo)
long long stage_w5_blocks(int nr, int nt, int np, int kplanes);
template <typename R>
void launch_stage_w5(const StageArgs<R>& a, int stage, int flux, int kplanes, hipStream_t s);
// rcp_fast / sqrt_fast of n doubles (accuracy diagnostics)
void launch_fast_math(const double* x, long long n, double* rcp, double* sq, hipStream_t s);
template <typename R>
void launch_finalize(DevClock* ck, const double* part, int nblocks, double cfl, int advance,
                     int log_on, const ProbeArgs& pa, const void* u, double* log,
                     hipStream_t s);

}  // namespace icr
