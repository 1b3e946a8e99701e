// icr_ensemble.hip -- batched ensemble of uneven runs on one GPU.
//
// Every run is a full solver (own grid, metric, maps, cone CMEs, clock and
// CFL dt).  One step of the ensemble walks four work lists that span all
// runs: boundary columns, stage-1 tiles, stage-2 tiles and one finalize per
// run.  The persistent kernel executes n steps in a single launch with a
// device-wide barrier between the lists; the batched mode launches one
// kernel per list.  Both run the same tile code as the single-run kernels,
// so each run's state is bit-identical to stepping it alone.
#include "icr_ensemble.hpp"

namespace icr {

// Items [0, n) split into 8 contiguous XCD slices; block b serves slice
// b % 8 with stride (blocks per XCD).
template <typename F>
__device__ __forceinline__ void for_items(int n, F&& f) {
  const int G = gridDim.x, b = blockIdx.x;
  const int xcd = b % NXCD, lb = b / NXCD, bpx = G / NXCD;
  const int lo = (int)((long long)xcd * n / NXCD), hi = (int)((long long)(xcd + 1) * n / NXCD);
  for (int it = lo + lb; it < hi; it += bpx) f(it);
}

__device__ __forceinline__ int find_run(const int* __restrict__ off, int n_runs, int item) {
  int lo = 0, hi = n_runs;  // off[lo] <= item < off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= item) lo = mid; else hi = mid;
  }
  return lo;
}

// Device-wide barrier (sense by generation count).  All blocks of the grid
// must be resident; a bounded spin turns a missing block into an error flag
// instead of a hang, and every block then leaves the kernel.
__device__ bool grid_sync(GridBar* gb, unsigned nblocks, long long spin_limit) {
  __shared__ int ok;
  __syncthreads();
  if (threadIdx.x == 0 && threadIdx.y == 0) {
    ok = 1;
    const unsigned g = __hip_atomic_load(&gb->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // release this block's writes (L2 write-back), then arrive
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned arrived = atomicAdd(&gb->count, 1u);
    if (arrived == nblocks - 1) {
      __hip_atomic_store(&gb->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      atomicAdd(&gb->gen, 1u);
    } else {
      long long n = 0;
      while (__hip_atomic_load(&gb->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
        __builtin_amdgcn_s_sleep(32);  // ~2000 cycles between polls of the shared line
        if (++n > spin_limit) {
          atomicExch(&gb->error, 1);
          ok = 0;
          break;
        }
      }
    }
    if (__hip_atomic_load(&gb->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) ok = 0;
    // acquire: later reads see every block's released writes
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  return ok != 0;
}

template <typename R>
__device__ __forceinline__ void bnd_item(const RunDesc<R>* runs, const EnsTables& e, int item) {
  const int r = find_run(e.bnd_off, e.n_runs, item);
  const RunDesc<R>& rd = runs[r];
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  const int q = (item - e.bnd_off[r]) * 256 + tid;
  const int plane = rd.bnd.nt * rd.bnd.np;
  if (q >= plane || !rd.clock->active) return;
  const int j = q % rd.bnd.nt, k = q / rd.bnd.nt;
  double w[NV];
  int in0, in1;
  boundary_prim(rd.bnd, rd.clock->t, j, k, w, &in0);
  for (int v = 0; v < NV; ++v) rd.ghost0[(long long)v * plane + q] = (R)w[v];
  boundary_prim(rd.bnd, rd.clock->t + rd.clock->dt, j, k, w, &in1);
  for (int v = 0; v < NV; ++v) rd.ghost1[(long long)v * plane + q] = (R)w[v];
  if (rd.tghost0) {  // tracer of the inner ghost cells: inside an inserted cone
    rd.tghost0[q] = (R)in0;
    rd.tghost1[q] = (R)in1;
  }
}

// Tracer item: 256 cells of one run, after that run's stage tiles.
template <typename R, int STAGE>
__device__ __forceinline__ void trc_item(const RunDesc<R>* runs, const EnsTables& e, int item,
                                         int step) {
  const int r = find_run(e.trc_off, e.n_runs, item);
  const RunDesc<R>& rd = runs[r];
  const int par = (rd.par + step) & 1;
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  const long long c = (long long)(item - e.trc_off[r]) * 256 + tid;
  tracer_cell<R, STAGE>(STAGE == 1 ? rd.t1[par] : rd.t2[par], c);
}

template <typename R, int FLUX, int LIM, int STAGE, bool FM>
__device__ __forceinline__ void stage_item(const RunDesc<R>* runs, const EnsTables& e, int item,
                                           int step, StageW<R, 64, 4>& smw,
                                           StageF<R, 64, 4>& smf) {
  const int r = find_run(e.tile_off, e.n_runs, item);
  const RunDesc<R>& rd = runs[r];
  const int local = item - e.tile_off[r];
  const int par = (rd.par + step) & 1;
  const int bx = local % rd.nbx, by = (local / rd.nbx) % rd.nby, bz = local / (rd.nbx * rd.nby);
  stage_tile<R, 64, 4, FLUX, LIM, STAGE, FM>(STAGE == 1 ? rd.s1[par] : rd.s2[par], rd.planes, bx,
                                             by, bz, local, smw, smf);
}

// WENO5: the 64 x 4 face-once tile with the three-cell halo (no tracer)
template <typename R, int FLUX, int STAGE>
__device__ __forceinline__ void stage_item_w5(const RunDesc<R>* runs, const EnsTables& e,
                                              int item, int step, StageW5<R>& sm) {
  const int r = find_run(e.tile_off, e.n_runs, item);
  const RunDesc<R>& rd = runs[r];
  const int local = item - e.tile_off[r];
  const int par = (rd.par + step) & 1;
  const int bx = local % rd.nbx, by = (local / rd.nbx) % rd.nby, bz = local / (rd.nbx * rd.nby);
  stage_tile_w5<R, FLUX, STAGE>(STAGE == 1 ? rd.s1[par] : rd.s2[par], rd.planes, bx, by, bz,
                                local, sm);
}

template <typename R>
__device__ __forceinline__ void fin_item(const RunDesc<R>* runs, int r) {
  const RunDesc<R>& rd = runs[r];
  ProbeArgs none{};
  finalize_run<R>(rd.clock, rd.partials, rd.nbx * rd.nby * rd.nbz, rd.cfl, 1, 0, none,
                  (const R*)nullptr, nullptr);
}

// FM: the passive tracer is on (stage tiles keep their face mass fluxes, a
// tracer list follows each stage list).
template <typename R, int FLUX, int LIM, bool FM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_ensemble(const RunDesc<R>* __restrict__ runs, EnsTables e, int nsteps) {
  const unsigned G = gridDim.x;
  __shared__ StageW<R, 64, 4> smw;
  __shared__ StageF<R, 64, 4> smf;
  for (int s = 0; s < nsteps; ++s) {
    for_items(e.n_bitems, [&](int it) { bnd_item<R>(runs, e, it); });
    if (!grid_sync(e.bar, G, e.spin_limit)) return;
    for_items(e.n_tiles, [&](int it) { stage_item<R, FLUX, LIM, 1, FM>(runs, e, it, s, smw, smf); });
    if (!grid_sync(e.bar, G, e.spin_limit)) return;
    if constexpr (FM) {
      for_items(e.n_titems, [&](int it) { trc_item<R, 1>(runs, e, it, s); });
      if (!grid_sync(e.bar, G, e.spin_limit)) return;
    }
    for_items(e.n_tiles, [&](int it) { stage_item<R, FLUX, LIM, 2, FM>(runs, e, it, s, smw, smf); });
    if (!grid_sync(e.bar, G, e.spin_limit)) return;
    if constexpr (FM) {
      for_items(e.n_titems, [&](int it) { trc_item<R, 2>(runs, e, it, s); });
      if (!grid_sync(e.bar, G, e.spin_limit)) return;
    }
    for_items(e.n_runs, [&](int r) { fin_item<R>(runs, r); });
    if (!grid_sync(e.bar, G, e.spin_limit)) return;
  }
}

template <typename R, int FLUX>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_ensemble_w5(const RunDesc<R>* __restrict__ runs, EnsTables e, int nsteps) {
  const unsigned G = gridDim.x;
  __shared__ StageW5<R> sm;
  for (int s = 0; s < nsteps; ++s) {
    for_items(e.n_bitems, [&](int it) { bnd_item<R>(runs, e, it); });
    if (!grid_sync(e.bar, G, e.spin_limit)) return;
    for_items(e.n_tiles, [&](int it) { stage_item_w5<R, FLUX, 1>(runs, e, it, s, sm); });
    if (!grid_sync(e.bar, G, e.spin_limit)) return;
    for_items(e.n_tiles, [&](int it) { stage_item_w5<R, FLUX, 2>(runs, e, it, s, sm); });
    if (!grid_sync(e.bar, G, e.spin_limit)) return;
    for_items(e.n_runs, [&](int r) { fin_item<R>(runs, r); });
    if (!grid_sync(e.bar, G, e.spin_limit)) return;
  }
}

// ---- batched mode: one launch per work list (grid = items) ---------------
template <typename R>
__global__ void __launch_bounds__(256) k_ens_bnd(const RunDesc<R>* __restrict__ runs, EnsTables e) {
  for_items(e.n_bitems, [&](int it) { bnd_item<R>(runs, e, it); });
}
template <typename R, int FLUX, int LIM, int STAGE, bool FM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_ens_stage(const RunDesc<R>* __restrict__ runs, EnsTables e, int step) {
  __shared__ StageW<R, 64, 4> smw;
  __shared__ StageF<R, 64, 4> smf;
  for_items(e.n_tiles,
            [&](int it) { stage_item<R, FLUX, LIM, STAGE, FM>(runs, e, it, step, smw, smf); });
}
template <typename R, int FLUX, int STAGE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_ens_stage_w5(const RunDesc<R>* __restrict__ runs, EnsTables e, int step) {
  __shared__ StageW5<R> sm;
  for_items(e.n_tiles, [&](int it) { stage_item_w5<R, FLUX, STAGE>(runs, e, it, step, sm); });
}
template <typename R, int STAGE>
__global__ void __launch_bounds__(256) k_ens_trc(const RunDesc<R>* __restrict__ runs, EnsTables e,
                                                 int step) {
  for_items(e.n_titems, [&](int it) { trc_item<R, STAGE>(runs, e, it, step); });
}
template <typename R>
__global__ void __launch_bounds__(256) k_ens_fin(const RunDesc<R>* __restrict__ runs, EnsTables e) {
  for_items(e.n_runs, [&](int r) { fin_item<R>(runs, r); });
}

__global__ void k_ens_clock_begin(DevClock* const* __restrict__ clocks, int n, double t_end) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  DevClock* ck = clocks[r];
  ck->t_end = t_end;
  ck->taken = 0;
  ck->active = ck->bad == BAD_NONE ? 1 : 0;
  set_next_dt(ck, ck->dt_cfl);
  if (ck->bad != BAD_NONE) ck->active = 0;
}

__global__ void k_ens_gather(DevClock* const* __restrict__ clocks, int n, DevClock* out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) out[r] = *clocks[r];
}

template <typename R, int FLUX, int LIM, bool FM>
static void ens_launch(const EnsLaunch& L, hipStream_t s) {
  const RunDesc<R>* runs = (const RunDesc<R>*)L.runs;
  const dim3 blk(64, 4);
  if (L.persistent) {
    hipLaunchKernelGGL((k_ensemble<R, FLUX, LIM, FM>), dim3(L.grid), blk, 0, s, runs, L.e,
                       L.nsteps);
    return;
  }
  auto items = [](int n) { return dim3((unsigned)((n + NXCD - 1) / NXCD * NXCD)); };
  for (int q = 0; q < L.nsteps; ++q) {
    hipLaunchKernelGGL(k_ens_bnd<R>, items(L.e.n_bitems), blk, 0, s, runs, L.e);
    hipLaunchKernelGGL((k_ens_stage<R, FLUX, LIM, 1, FM>), items(L.e.n_tiles), blk, 0, s, runs,
                       L.e, q);
    if (FM) hipLaunchKernelGGL((k_ens_trc<R, 1>), items(L.e.n_titems), blk, 0, s, runs, L.e, q);
    hipLaunchKernelGGL((k_ens_stage<R, FLUX, LIM, 2, FM>), items(L.e.n_tiles), blk, 0, s, runs,
                       L.e, q);
    if (FM) hipLaunchKernelGGL((k_ens_trc<R, 2>), items(L.e.n_titems), blk, 0, s, runs, L.e, q);
    hipLaunchKernelGGL(k_ens_fin<R>, items(L.e.n_runs), blk, 0, s, runs, L.e);
  }
}

template <typename R, int FLUX>
static void ens_launch_w5(const EnsLaunch& L, hipStream_t s) {
  const RunDesc<R>* runs = (const RunDesc<R>*)L.runs;
  const dim3 blk(64, 4);
  if (L.persistent) {
    hipLaunchKernelGGL((k_ensemble_w5<R, FLUX>), dim3(L.grid), blk, 0, s, runs, L.e, L.nsteps);
    return;
  }
  auto items = [](int n) { return dim3((unsigned)((n + NXCD - 1) / NXCD * NXCD)); };
  for (int q = 0; q < L.nsteps; ++q) {
    hipLaunchKernelGGL(k_ens_bnd<R>, items(L.e.n_bitems), blk, 0, s, runs, L.e);
    hipLaunchKernelGGL((k_ens_stage_w5<R, FLUX, 1>), items(L.e.n_tiles), blk, 0, s, runs, L.e, q);
    hipLaunchKernelGGL((k_ens_stage_w5<R, FLUX, 2>), items(L.e.n_tiles), blk, 0, s, runs, L.e, q);
    hipLaunchKernelGGL(k_ens_fin<R>, items(L.e.n_runs), blk, 0, s, runs, L.e);
  }
}

template <typename R, int FLUX, int LIM>
static void ens_launch_fm(const EnsLaunch& L, hipStream_t s) {
  if (L.tracer) ens_launch<R, FLUX, LIM, true>(L, s);
  else ens_launch<R, FLUX, LIM, false>(L, s);
}

template <typename R, int FLUX>
static void ens_launch_lim(const EnsLaunch& L, hipStream_t s) {
  if (L.lim == LIM_MINMOD) ens_launch_fm<R, FLUX, LIM_MINMOD>(L, s);
  else if (L.lim == LIM_WENO5) ens_launch_w5<R, FLUX>(L, s);  // the host rejects the tracer
  else ens_launch_fm<R, FLUX, LIM_MC>(L, s);
}

template <typename R>
static void ens_dispatch(const EnsLaunch& L, hipStream_t s) {
  if (L.flux == FLUX_TVDLF) ens_launch_lim<R, FLUX_TVDLF>(L, s);
  else if (L.flux == FLUX_HLLD) ens_launch_lim<R, FLUX_HLLD>(L, s);
  else ens_launch_lim<R, FLUX_HLL>(L, s);
}

void launch_ensemble(const EnsLaunch& L, bool f32, hipStream_t s) {
  if (f32) ens_dispatch<float>(L, s);
  else ens_dispatch<double>(L, s);
}

void launch_ens_clock_begin(DevClock* const* clocks, int n, double t_end, hipStream_t s) {
  hipLaunchKernelGGL(k_ens_clock_begin, dim3((n + 63) / 64), dim3(64), 0, s, clocks, n, t_end);
}

void launch_ens_gather(DevClock* const* clocks, int n, DevClock* out, hipStream_t s) {
  hipLaunchKernelGGL(k_ens_gather, dim3((n + 63) / 64), dim3(64), 0, s, clocks, n, out);
}

template <typename R, int FLUX, int LIM>
static const void* ens_fn(bool tracer) {
  return tracer ? reinterpret_cast<const void*>(&k_ensemble<R, FLUX, LIM, true>)
                : reinterpret_cast<const void*>(&k_ensemble<R, FLUX, LIM, false>);
}

template <typename R>
static const void* ens_fn_r(int flux, int lim, bool tracer) {
  if (lim == LIM_WENO5) {
    if (flux == FLUX_TVDLF) return reinterpret_cast<const void*>(&k_ensemble_w5<R, FLUX_TVDLF>);
    if (flux == FLUX_HLLD) return reinterpret_cast<const void*>(&k_ensemble_w5<R, FLUX_HLLD>);
    return reinterpret_cast<const void*>(&k_ensemble_w5<R, FLUX_HLL>);
  }
  const bool mm = lim == LIM_MINMOD;
  if (flux == FLUX_TVDLF)
    return mm ? ens_fn<R, FLUX_TVDLF, LIM_MINMOD>(tracer) : ens_fn<R, FLUX_TVDLF, LIM_MC>(tracer);
  if (flux == FLUX_HLLD)
    return mm ? ens_fn<R, FLUX_HLLD, LIM_MINMOD>(tracer) : ens_fn<R, FLUX_HLLD, LIM_MC>(tracer);
  return mm ? ens_fn<R, FLUX_HLL, LIM_MINMOD>(tracer) : ens_fn<R, FLUX_HLL, LIM_MC>(tracer);
}

int ensemble_blocks_per_cu(bool f32, int flux, int lim, bool tracer) {
  int nb = 0;
  const void* fn = f32 ? ens_fn_r<float>(flux, lim, tracer) : ens_fn_r<double>(flux, lim, tracer);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 256, 0) != hipSuccess) return 0;
  return nb;
}

}  // namespace icr
