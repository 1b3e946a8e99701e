// icr_stage_lds.hip -- single-run launches of the face-once stage kernel
// and the finalize kernel (device code in icr_stage_lds.hpp).
#include "icr_stage_lds.hpp"
#include "icr_stage_w5.hpp"

namespace icr {

#ifndef ICR_LDS_WAVES
#define ICR_LDS_WAVES 2
#endif

template <typename R, int TR, int TT, int FLUX, int LIM, int STAGE, bool FM>
__global__ void __launch_bounds__(TR* TT) __attribute__((amdgpu_waves_per_eu(ICR_LDS_WAVES)))
k_stage_lds(StageArgs<R> a, int kplanes) {
  const int nbx = gridDim.x, nby = gridDim.y;
  const int nb = nbx * nby * gridDim.z;
  const int b = (blockIdx.z * nby + blockIdx.y) * nbx + blockIdx.x;
  const int tile = xcd_tile(b, nb);
  __shared__ StageW<R, TR, TT> smw;
  __shared__ StageF<R, TR, TT> smf;
  stage_tile<R, TR, TT, FLUX, LIM, STAGE, FM>(a, kplanes, tile % nbx, (tile / nbx) % nby,
                                              tile / (nbx * nby), tile, smw, smf);
}

template <typename R, int TR, int TT, int FLUX, int LIM, bool FM>
static void launch_lds_t(const StageArgs<R>& a, int stage, int kplanes, hipStream_t s) {
  constexpr int TI = tile_cells_r(TR);
  const dim3 grid((a.nr + TI - 1) / TI, (a.nt + TT - 1) / TT, (a.np + kplanes - 1) / kplanes);
  const dim3 blk(TR, TT);
  if (stage == 1)
    hipLaunchKernelGGL((k_stage_lds<R, TR, TT, FLUX, LIM, 1, FM>), grid, blk, 0, s, a, kplanes);
  else
    hipLaunchKernelGGL((k_stage_lds<R, TR, TT, FLUX, LIM, 2, FM>), grid, blk, 0, s, a, kplanes);
}

template <typename R, int TR, int TT, bool FM>
static void launch_lds_tile(const StageArgs<R>& a, int stage, int flux, int lim, int kplanes,
                            hipStream_t s) {
  if (flux == FLUX_TVDLF) {
    if (lim == LIM_MINMOD)
      launch_lds_t<R, TR, TT, FLUX_TVDLF, LIM_MINMOD, FM>(a, stage, kplanes, s);
    else
      launch_lds_t<R, TR, TT, FLUX_TVDLF, LIM_MC, FM>(a, stage, kplanes, s);
  } else if (flux == FLUX_HLLD) {
    if (lim == LIM_MINMOD)
      launch_lds_t<R, TR, TT, FLUX_HLLD, LIM_MINMOD, FM>(a, stage, kplanes, s);
    else
      launch_lds_t<R, TR, TT, FLUX_HLLD, LIM_MC, FM>(a, stage, kplanes, s);
  } else {
    if (lim == LIM_MINMOD)
      launch_lds_t<R, TR, TT, FLUX_HLL, LIM_MINMOD, FM>(a, stage, kplanes, s);
    else
      launch_lds_t<R, TR, TT, FLUX_HLL, LIM_MC, FM>(a, stage, kplanes, s);
  }
}

// With the passive tracer (a.fmass set) only the 64 x 4 tile is built with
// the mass-flux stores; the solver keeps tile_r = 64 in that case.
template <typename R>
void launch_stage_lds(const StageArgs<R>& a, int stage, int flux, int lim, int tile_r,
                      int kplanes, hipStream_t s) {
  if (a.fmass)
    launch_lds_tile<R, 64, 4, true>(a, stage, flux, lim, kplanes, s);
  else if (tile_r == 32)
    launch_lds_tile<R, 32, 8, false>(a, stage, flux, lim, kplanes, s);
  else
    launch_lds_tile<R, 64, 4, false>(a, stage, flux, lim, kplanes, s);
}
template void launch_stage_lds<double>(const StageArgs<double>&, int, int, int, int, int,
                                       hipStream_t);
template void launch_stage_lds<float>(const StageArgs<float>&, int, int, int, int, int,
                                      hipStream_t);

// WENO5: the face-once tile with a three-cell halo (64 x 4 threads, 58
// cells along r per row)
template <typename R, int FLUX, int STAGE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(ICR_LDS_WAVES)))
k_stage_w5(StageArgs<R> a, int kplanes) {
  const int nbx = gridDim.x, nby = gridDim.y;
  const int nb = nbx * nby * gridDim.z;
  const int b = (blockIdx.z * nby + blockIdx.y) * nbx + blockIdx.x;
  const int tile = xcd_tile(b, nb);
  __shared__ StageW5<R> sm;
  stage_tile_w5<R, FLUX, STAGE>(a, kplanes, tile % nbx, (tile / nbx) % nby, tile / (nbx * nby),
                                tile, sm);
}

template <typename R, int FLUX>
static void launch_w5_t(const StageArgs<R>& a, int stage, int kplanes, hipStream_t s) {
  const dim3 grid((a.nr + W5_TI - 1) / W5_TI, (a.nt + W5_TT - 1) / W5_TT,
                  (a.np + kplanes - 1) / kplanes);
  const dim3 blk(W5_TR, W5_TT);
  if (stage == 1)
    hipLaunchKernelGGL((k_stage_w5<R, FLUX, 1>), grid, blk, 0, s, a, kplanes);
  else
    hipLaunchKernelGGL((k_stage_w5<R, FLUX, 2>), grid, blk, 0, s, a, kplanes);
}

template <typename R>
void launch_stage_w5(const StageArgs<R>& a, int stage, int flux, int kplanes, hipStream_t s) {
  if (flux == FLUX_TVDLF) launch_w5_t<R, FLUX_TVDLF>(a, stage, kplanes, s);
  else if (flux == FLUX_HLLD) launch_w5_t<R, FLUX_HLLD>(a, stage, kplanes, s);
  else launch_w5_t<R, FLUX_HLL>(a, stage, kplanes, s);
}
template void launch_stage_w5<double>(const StageArgs<double>&, int, int, int, hipStream_t);
template void launch_stage_w5<float>(const StageArgs<float>&, int, int, int, hipStream_t);

long long stage_w5_blocks(int nr, int nt, int np, int kplanes) {
  return (long long)((nr + W5_TI - 1) / W5_TI) * ((nt + W5_TT - 1) / W5_TT) *
         ((np + kplanes - 1) / kplanes);
}

long long stage_lds_blocks(int nr, int nt, int np, int tile_r, int kplanes) {
  const int tt = 256 / tile_r, ti = tile_cells_r(tile_r);
  return (long long)((nr + ti - 1) / ti) * ((nt + tt - 1) / tt) *
         ((np + kplanes - 1) / kplanes);
}

template <typename R>
__global__ void __launch_bounds__(256) k_finalize(DevClock* ck, const double* __restrict__ part,
                                                  int nblocks, double cfl, int advance,
                                                  int log_on, ProbeArgs pa,
                                                  const R* __restrict__ u,
                                                  double* __restrict__ log) {
  finalize_run<R>(ck, part, nblocks, cfl, advance, log_on, pa, u, log);
}

template <typename R>
void launch_finalize(DevClock* ck, const double* part, int nblocks, double cfl, int advance,
                     int log_on, const ProbeArgs& pa, const void* u, double* log,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_finalize<R>, dim3(1), dim3(256), 0, s, ck, part, nblocks, cfl, advance,
                     log_on, pa, (const R*)u, log);
}
template void launch_finalize<double>(DevClock*, const double*, int, double, int, int,
                                      const ProbeArgs&, const void*, double*, hipStream_t);
template void launch_finalize<float>(DevClock*, const double*, int, double, int, int,
                                     const ProbeArgs&, const void*, double*, hipStream_t);

}  // namespace icr
