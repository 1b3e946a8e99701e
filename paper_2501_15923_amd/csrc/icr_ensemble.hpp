// icr_ensemble.hpp -- device tables of the batched ensemble.
#pragma once
#include "icr_stage_lds.hpp"
#include "icr_stage_w5.hpp"

namespace icr {

struct GridBar {
  unsigned count;  // blocks arrived at the current barrier
  unsigned gen;    // barrier generation
  int error;       // 1: a bounded wait expired (a block was not resident)
  int pad;
};

// One run of the ensemble: stage arguments for both parities of the source
// buffer (stage 1 reads U[p] and writes U[2]; stage 2 reads U[2], U[p] and
// writes U[p^1]), its boundary data, clock, partial slots and tile grid.
template <typename R>
struct RunDesc {
  StageArgs<R> s1[2], s2[2];
  TracerArgs<R> t1[2], t2[2];  // passive tracer stages (used when the ensemble has it)
  BndArgs bnd;
  R* ghost0;
  R* ghost1;
  R* tghost0;  // tau of the inner ghost cells at the two stage times (tracer on)
  R* tghost1;
  DevClock* clock;
  double* partials;
  int nbx, nby, nbz, planes;
  int par;  // parity of the current state buffer when the launch starts
  double cfl;
};

struct EnsTables {
  int n_runs;
  int n_tiles;          // stage tiles over all runs
  int n_bitems;         // boundary items of 256 columns over all runs
  int n_titems;         // tracer items of 256 cells over all runs (0: tracer off)
  const int* tile_off;  // [n_runs + 1] prefix sums of tiles
  const int* bnd_off;   // [n_runs + 1] prefix sums of boundary items
  const int* trc_off;   // [n_runs + 1] prefix sums of tracer items
  GridBar* bar;
  long long spin_limit;
};

struct EnsLaunch {
  const void* runs;  // RunDesc<R>[n_runs] on the device
  EnsTables e;
  int persistent, grid, nsteps, flux, lim, tracer;
};

void launch_ensemble(const EnsLaunch& L, bool f32, hipStream_t s);
void launch_ens_clock_begin(DevClock* const* clocks, int n, double t_end, hipStream_t s);
void launch_ens_gather(DevClock* const* clocks, int n, DevClock* out, hipStream_t s);
int ensemble_blocks_per_cu(bool f32, int flux, int lim, bool tracer);

}  // namespace icr
