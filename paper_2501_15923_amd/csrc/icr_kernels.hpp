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
};

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

template <typename R>
Metric<R> metric_view(const R* base, int nr, int nt, double dth);

void launch_metric(const MetricArgs& a, void* mr, bool f32, hipStream_t s);
void launch_boundary(const BndArgs& a, const DevClock* ck, void* g1, void* g2, bool f32,
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
template <typename R>
void launch_import(const double* in, void* u, long long n, int kind, const Scale& sc, double gam,
                   hipStream_t s);
template <typename R>
void launch_export(const void* u, double* out, long long n, int kind, const Scale& sc, double gam,
                   hipStream_t s);
template <typename R>
void launch_probe_sample(const ProbeArgs& a, const DevClock* ck, const void* u, double* out,
                         hipStream_t s);
template <typename R>
void launch_probe_log(const ProbeArgs& a, DevClock* ck, const void* u, double* log,
                      hipStream_t s);

}  // namespace icr
