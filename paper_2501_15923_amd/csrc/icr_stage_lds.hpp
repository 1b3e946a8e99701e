// icr_stage_lds.hpp -- device code of the face-once stage (shared by the
// single-run kernels and the ensemble kernels, so that both execute the same
// arithmetic).
//
// One RK2 stage of the finite-volume update (Sect. 2 Eqs. 1-6) with every
// face flux computed exactly once:
//   - a block of TR x TT threads marches along phi over a chunk of planes;
//     each row of TR lanes covers TR - 4 cells of the tile plus the two-cell
//     r halo on either side (the halo lanes load and convert their cells
//     like every other lane, so the r halo costs no extra loads);
//   - per plane the primitives of the tile's rows plus a two-row theta halo
//     sit in LDS; r- and theta-face fluxes go to LDS and are shared by the
//     two cells of each face;
//   - the phi direction is carried in registers: each thread keeps the
//     primitives of planes k-1 .. k+2 of its own column and the flux of
//     face k-1/2 from the previous plane.
// Lanes run along r, so global loads and stores are coalesced (state layout
// [8][n_phi][n_theta][n_r]).  Stage 2 also forms the per-block partials of
// the next CFL dt, of the relaxation residual and of the validity flag; a
// one-block finalize reduces them in a fixed order.
#pragma once
#include "icr_kernels.hpp"

namespace icr {


template <typename R, bool FAST>
__device__ __forceinline__ void load_cons_prim(const StageArgs<R>& a, unsigned c, R (&w)[NV]) {
  R u[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) u[v] = ldg(a.uin + v * a.ncell, c);
  cons2prim<R, FAST>(u, w, a.gm1);
}

__device__ __forceinline__ int wrap_phi(int k, int np) { return ((k % np) + np) % np; }

// Face states of face m-1/2 from four LDS values per variable (p0..p3 =
// cells m-2 .. m+1), then the numerical flux.
template <typename R, int N, int FLUX, int LIM>
__device__ __forceinline__ void lds_face(const R* base, int stride, R gam, R igm1, R (&f)[NV],
                                         int vstride) {
  R wl[NV], wr[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const R* q = base + v * vstride;
    const R p0 = q[0], p1 = q[stride], p2 = q[2 * stride], p3 = q[3 * stride];
    wl[v] = p1 + R(0.5) * limiter<R, LIM, true>(p1 - p0, p2 - p1);
    wr[v] = p2 - R(0.5) * limiter<R, LIM, true>(p2 - p1, p3 - p2);
  }
  face_flux<R, N, FLUX, true>(wl, wr, gam, igm1, f);
}

// One tile (bx, by, bz) of one run: (TR - 4) x TT columns, planes
// bz*kplanes ..; stage-2 partials go to slot pslot.  Called by the
// single-run kernel and by the ensemble kernels, so both execute the same
// code.
// LDS of one tile, indexed by lane along r (lane l holds cell i0 + l - 2):
// primitives of rows -2 .. TT+1 (StageW), the flux of r face i-1/2 at the
// lane of cell i and the flux of theta face j-1/2 at row j (0 .. TT)
// (StageF).  Two separate LDS objects, declared once per kernel and passed
// to stage_tile: the compiler can then tell that the update's flux reads do
// not touch the rows the stage-2 LDS-DMA copies are landing in, and does not
// wait for those copies before them.
template <typename R, int TR, int TT>
struct alignas(16) StageW {
  R sW[NV][TT + 4][TR];
};
template <typename R, int TR, int TT>
struct alignas(16) StageF {
  R sFr[NV][TT][TR];
  R sFt[NV][TT + 1][TR];
  // the metric factors of the tile's cells, loaded once per block: per-r
  // arrays at each lane's cell, per-theta arrays at each row's cell (the
  // update then reads them from LDS instead of loading them every plane)
  R mr[MR_N][TR];
  R mt[MT_N][TT];
};

// Cell-metric accessor over the tile's LDS copy (lane li, row lj).
template <typename R, int TR, int TT>
struct LdsCellMetric {
  const StageF<R, TR, TT>& f;
  int li, lj;
  R ilth_;
  __device__ __forceinline__ R r(int a) const { return f.mr[a][li]; }
  __device__ __forceinline__ R t(int a) const { return f.mt[a][lj]; }
  __device__ __forceinline__ R ilth() const { return ilth_; }
};

// Stage-2 theta-halo copies: a halo region is the two rows on one side of
// the tile (2 TR values of one variable, contiguous in LDS), copied by wave
// instructions of 64 lanes x dw bytes (16 where a region is a multiple of
// 1 KiB, else 4); instruction n of a plane covers chunk n % ipr of region
// (n / ipr) % 2 of variable n / (2 ipr), and wave w issues n = w, w + nw,
// ...  Each wave keeps the byte offsets of the first ppw of its (region,
// chunk) pairs; this checks that they repeat with period ppw.
// One LDS-DMA copy: every lane moves BYTES bytes from its own global
// address to dst + BYTES * lane (dst is the same for the whole wave).
template <int BYTES>
__device__ __forceinline__ void lds_dma(const char* src, char* dst) {
  static_assert(BYTES == 16 || BYTES == 4, "LDS-DMA copy width");
  auto g = (const __attribute__((address_space(1))) void*)src;
  auto l = (__attribute__((address_space(3))) void*)dst;
  if constexpr (BYTES == 16)
    __builtin_amdgcn_global_load_lds(g, l, 16, 0, 0);
  else
    __builtin_amdgcn_global_load_lds(g, l, 4, 0, 0);
}

constexpr bool dma_pairs_periodic(int nw, int ipr, int per_wave, int ppw) {
  for (int w = 0; w < nw; ++w)
    for (int m = 0; m < per_wave; ++m) {
      const int n = w + nw * m, q = w + nw * (m % ppw);
      if (n % ipr != q % ipr || (n / ipr) % 2 != (q / ipr) % 2) return false;
    }
  return true;
}

template <typename R, int TR, int TT, int FLUX, int LIM, int STAGE, bool FM = false>
__device__ __forceinline__ void stage_tile(const StageArgs<R>& a, int kplanes, int bx, int by,
                                           int bz, int pslot, StageW<R, TR, TT>& smw,
                                           StageF<R, TR, TT>& smf) {
  constexpr int NT = TR * TT;
  constexpr int TI = tile_cells_r(TR);
  constexpr int WT = TT + 4;
  auto& sW = smw.sW;
  auto& sFr = smf.sFr;
  auto& sFt = smf.sFt;

  const int ti = threadIdx.x, tj = threadIdx.y, tid = tj * TR + ti;
  const int i0 = bx * TI, j0 = by * TT, k0 = bz * kplanes;
  const int nr = a.nr, nt = a.nt, np = a.np;
  const int kend = k0 + kplanes < np ? k0 + kplanes : np;
  const int i = i0 + ti - 2, j = j0 + tj;  // this lane's cell
  const bool inner = ti >= 2 && ti < TR - 2;
  const bool valid = inner && i < nr && j < nt;
  // column of the own phi ring: the cell itself, the last cell beyond r_out;
  // below r_in cell 0, or under the asymm rule the mirror cell -1 - i, whose
  // transverse primitives the ghost takes negated
  const int ic = i < 0 ? (a.asymm ? (-1 - i < nr ? -1 - i : nr - 1) : 0)
                       : (i < nr ? i : nr - 1);
  const int jc = j < nt ? j : nt - 1;
  const int active = a.clock->active;
  // cell offsets within one variable's array (32-bit: below 2^29 cells)
  const unsigned colbase = (unsigned)(jc * nr + ic);  // + k * nt * nr
  // own-column loads: rows past the last colatitude mirror it (they serve
  // as ghost rows of the last active row's upper theta face); cells below
  // r_in (halo lanes of the first tile) come from the inner ghost, cells
  // beyond r_out repeat the last cell
  bool flipj;
  const int mj = mirror_row(j, nt, flipj);
  const unsigned lbase = (unsigned)(mj * nr + ic);
  const bool lghost = i < 0;
  const unsigned plane_cells = (unsigned)(nt * nr);
  const long long gplane = (long long)nt * np;
  // The ring of the first tile's two halo lanes below r_in holds cell 0 (or
  // the mirror cell); those lanes put the inner ghost into LDS instead (see
  // below).
  // the next plane's own-column state is loaded one plane ahead (raw
  // conserved values in uring) and converted when the phi face needs it
  auto own_raw = [&](int k, R (&u)[NV]) {
    const unsigned c = (unsigned)wrap_phi(k, np) * plane_cells + lbase;
#pragma unroll
    for (int v = 0; v < NV; ++v) u[v] = ldg(a.uin + v * a.ncell, c);
  };
  auto own_cvt = [&](const R (&u)[NV], R (&w)[NV]) {
    cons2prim<R, true>(u, w, a.gm1);
    if (flipj) flip_theta(w);
  };
  auto load_own = [&](int k, R (&w)[NV]) {
    load_cons_prim<R, true>(a, (unsigned)wrap_phi(k, np) * plane_cells + lbase, w);
    if (flipj) flip_theta(w);
  };

  if (!active) {
    if (STAGE == 2 && valid)
      for (int k = k0; k < kend; ++k) {
        const unsigned c = (unsigned)k * plane_cells + colbase;
#pragma unroll
        for (int v = 0; v < NV; ++v) stg(a.uout + v * a.ncell, c, ldg(a.un + v * a.ncell, c));
      }
    return;
  }

  // metric factors of the tile into LDS (visible after the first plane
  // barrier; the first use is after it).  A block that runs several tiles
  // (ensembles) first waits until every wave has left the previous tile.
  __syncthreads();
  // (array indices are compile-time constants after unrolling, so that the
  // metric pointers stay kernel arguments)
  for (int l = tid; l < TR; l += NT) {
    const int ii = i0 + l - 2;
    const int icl = ii < 0 ? (a.asymm ? (-1 - ii < nr ? -1 - ii : nr - 1) : 0)
                           : (ii < nr ? ii : nr - 1);
#pragma unroll
    for (int arr = 0; arr < MR_N; ++arr) smf.mr[arr][l] = ldg(metric_r(a.m, arr), (unsigned)icl);
  }
  for (int row = tid; row < TT; row += NT) {
    const int jr = j0 + row < nt ? j0 + row : nt - 1;
#pragma unroll
    for (int arr = 0; arr < MT_N; ++arr) smf.mt[arr][row] = ldg(metric_t(a.m, arr), (unsigned)jr);
  }
  const LdsCellMetric<R, TR, TT> cm{smf, ti, tj, a.m.ilth};
  // the stage's dt, read once: a global load inside the update would make
  // it wait for the stage-2 halo copies issued before it
  const R dt = (R)a.clock->dt;

  // phi ring of the own column: at the top of iteration k, wa = W(k-1),
  // wb = W(k), wc = W(k+1) and fcar = flux of face k-1/2.  Iteration k0-1
  // only forms fcar, through the same code as every later phi face.
  R wa[NV], wb[NV], wc[NV], fcar[NV];
  load_own(k0 - 2, wa);
  load_own(k0 - 1, wb);
  load_own(k0, wc);
  R uring[NV];
  own_raw(k0 + 1, uring);
#pragma unroll
  for (int v = 0; v < NV; ++v) fcar[v] = R(0);

  // Stage 1 (PF): this thread's theta-halo item is the same (row, lane) of
  // every plane, and the next plane's item is loaded into registers while
  // the current plane is processed.  Stage 2 (DMA) has no registers to
  // spare: the next plane's halo rows are copied global -> LDS by the LDS-DMA
  // loads, issued after the plane's face barrier (nothing reads sW until the
  // next plane barrier), so they travel while the plane is updated; after
  // the next plane barrier each thread converts its halo cell to primitives
  // in place.  Those copies take, for a halo cell below r_in or beyond
  // r_out, the clamped cell of its row: such cells only feed the theta
  // faces of halo lanes, which the update never reads.
  constexpr bool PF = STAGE == 1;
  constexpr bool DMA = STAGE == 2;
  static_assert(4 * TR <= NT, "at most one theta-halo item per thread");
  const bool hv = tid < 4 * TR;
  const int hrow = tid / TR, hl = tid - hrow * TR;
  const int hjj = hrow < 2 ? hrow - 2 : TT + hrow - 2;
  const int hgi = i0 + hl - 2;
  bool hflip;
  const int hgj = mirror_row(j0 + hjj, nt, hflip);
  const bool hghost = hgi < 0;  // below r_in: inner ghost primitives
  const unsigned hoff = (unsigned)(hgj * nr + (hgi < 0 ? 0 : (hgi < nr ? hgi : nr - 1)));
  auto halo_raw = [&](int k, R (&w)[NV]) {
    if (hghost) {
#pragma unroll
      for (int v = 0; v < NV; ++v) w[v] = ldg(a.ghost + v * gplane, (unsigned)(k * nt + hgj));
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) w[v] = ldg(a.uin + v * a.ncell, (unsigned)k * plane_cells + hoff);
    }
  };
  auto halo_put = [&](const R (&raw)[NV]) {
    R w[NV];
    if (hghost) {
#pragma unroll
      for (int v = 0; v < NV; ++v) w[v] = raw[v];
    } else {
      cons2prim<R, true>(raw, w, a.gm1);
    }
    if (hflip) flip_theta(w);
#pragma unroll
    for (int v = 0; v < NV; ++v) sW[v][hjj + 2][hl] = w[v];
  };
  R hraw[NV];
  if (PF && hv && k0 < kend) halo_raw(k0, hraw);

  // (the copies need n_r >= 2: a 16-byte copy takes two neighbouring cells
  // of a row; with fewer cells stage 2 loads its halo after the barrier)
  constexpr int NW = NT / 64;                              // waves per block
  constexpr int RB = 2 * TR * (int)sizeof(R);              // bytes of a halo region
  constexpr int DW = RB % 1024 == 0 ? 16 : 4;              // bytes per lane and copy
  constexpr int IPR = RB / (64 * DW) > 0 ? RB / (64 * DW) : 1;  // copies per region
  constexpr int NINS = NV * 2 * IPR;                       // per plane
  constexpr int PPW = 2 * IPR > NW ? 2 * IPR / NW : 1;     // (region, chunk) pairs per wave
  constexpr int SPAN = DW / (int)sizeof(R) > 1 ? DW / (int)sizeof(R) : 1;  // cells per copy
  static_assert(!DMA || (NT % 64 == 0 && RB % (64 * DW) == 0 && NINS % NW == 0 &&
                         dma_pairs_periodic(NW, IPR, NINS / NW, PPW) && SPAN <= 2 &&
                         tile_cells_r(TR) % 2 == 0),
                "theta-halo DMA layout");
  const bool dma_on = DMA && nr >= 2;  // uniform
  const int wv = __builtin_amdgcn_readfirstlane(tid) >> 6;  // wave index (uniform)
  unsigned doff[PPW];  // byte offset in a plane of this lane's dw bytes, per pair
  if constexpr (DMA) {
    const int lane = tid & 63;
#pragma unroll
    for (int p = 0; p < PPW; ++p) {
      const int n = wv + NW * p;
      const int c = n % IPR, reg = (n / IPR) % 2;
      const int b = (c * 64 + lane) * DW;
      const int e = b / (int)sizeof(R);  // first value of this lane's copy
      const int rr = e / TR, l = e - rr * TR;
      bool fl;
      const int gj = mirror_row(j0 + (reg ? TT + rr : rr - 2), nt, fl);
      // clamped into the row; a two-cell copy keeps both cells in the row
      int gi = i0 + l - 2;
      gi = gi < 0 ? 0 : (gi <= nr - SPAN ? gi : nr - SPAN);
      doff[p] = (unsigned)(gj * nr + gi) * (unsigned)sizeof(R) + (unsigned)(b % (int)sizeof(R));
    }
  }
  auto dma_halo = [&](int k) {
    const unsigned kb = (unsigned)k * plane_cells * (unsigned)sizeof(R);
#pragma unroll
    for (int m = 0; m < NINS / NW; ++m) {
      const int n = wv + NW * m;
      const int c = n % IPR, reg = (n / IPR) % 2, v = n / (2 * IPR);
      const char* src = reinterpret_cast<const char*>(a.uin + (size_t)v * a.ncell) + kb +
                        doff[m % PPW];
      char* dst = reinterpret_cast<char*>(&sW[v][reg ? TT + 2 : 0][0]) + c * 64 * DW;
      lds_dma<DW>(src, dst);
    }
  };
  if constexpr (DMA) {
    if (dma_on && k0 < kend) dma_halo(k0);
  }

  double lam = 0.0, s1 = 0.0, s0 = 0.0;
  int bad = BAD_NONE;

  for (int k = k0 - 1; k < kend; ++k) {
    const bool body = k >= k0;  // uniform over the block
    const unsigned kbase = (unsigned)k * plane_cells;
    if (body) {
      // stage 2: this wave's halo copies have landed (s_waitcnt vmcnt(0));
      // the barrier then makes every wave's copies visible
      if constexpr (DMA) {
        if (dma_on) __builtin_amdgcn_s_waitcnt(0x3f70);
      }
      __syncthreads();  // the previous plane's LDS reads are complete
      if (lghost) {  // inner ghost (primitives) at this lane's row
        R w[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) w[v] = ldg(a.ghost + v * gplane, (unsigned)(k * nt + mj));
        if (flipj) flip_theta(w);
        if (a.asymm) {  // wb: the mirror cell's primitives (already flipped)
          w[2] = -wb[2];
          w[3] = -wb[3];
          w[6] = -wb[6];
          w[7] = -wb[7];
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) sW[v][tj + 2][ti] = w[v];
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) sW[v][tj + 2][ti] = wb[v];
      }
      // theta halo: rows -2, -1, TT, TT + 1 over all TR lanes
      if constexpr (PF) {
        if (hv) {
          halo_put(hraw);
          if (k + 1 < kend) halo_raw(k + 1, hraw);  // in flight during this plane
        }
      } else if (dma_on) {
        if (hv) {  // conserved -> primitive in place
          R u[NV], w[NV];
          // a two-cell copy starts at an even lane (an even cell, the tile
          // start being even): at the end of a row of odd length it was
          // shifted back into the row, so the even lane of the last cell got
          // its left neighbour; reload that one cell
          if (SPAN == 2 && hgi == nr - 1 && (hl & 1) == 0 && hl >= 2 && hl < TR - 2) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
              u[v] = ldg(a.uin + v * a.ncell, kbase + (unsigned)(hgj * nr + hgi));
          } else {
#pragma unroll
            for (int v = 0; v < NV; ++v) u[v] = sW[v][hjj + 2][hl];
          }
          cons2prim<R, true>(u, w, a.gm1);
          if (hflip) flip_theta(w);
#pragma unroll
          for (int v = 0; v < NV; ++v) sW[v][hjj + 2][hl] = w[v];
        }
      } else {
        for (int h = tid; h < 4 * TR; h += NT) {
          const int row = h / TR, l = h - row * TR;
          const int jj = row < 2 ? row - 2 : TT + row - 2;
          const int gi = i0 + l - 2;
          bool flip;
          const int gj = mirror_row(j0 + jj, nt, flip);
          R w[NV];
          if (gi < 0) {
            const unsigned g = (unsigned)(k * nt + gj);
#pragma unroll
            for (int v = 0; v < NV; ++v) w[v] = ldg(a.ghost + v * gplane, g);
          } else {
            load_cons_prim<R, true>(a, kbase + (unsigned)(gj * nr + (gi < nr ? gi : nr - 1)), w);
          }
          if (flip) flip_theta(w);
#pragma unroll
          for (int v = 0; v < NV; ++v) sW[v][jj + 2][l] = w[v];
        }
      }
      __syncthreads();
      // r face i-1/2 and theta face j-1/2 at every lane (the update reads
      // the r faces of lanes 2 .. TR-2, the last being the tile's upper r
      // face, and the theta faces of the inner lanes; the others are never
      // read, and lanes 0, 1 and TR-1 read neighbouring LDS rows for their
      // r face), then the tile's upper theta face of every inner lane
      constexpr int VS = WT * TR;
      {
        R f[NV];
        lds_face<R, 1, FLUX, LIM>(&sW[0][tj + 2][ti] - 2, 1, a.gam, a.igm1, f, VS);
#pragma unroll
        for (int v = 0; v < NV; ++v) sFr[v][tj][ti] = f[v];
      }
      {
        R f[NV];
        lds_face<R, 2, FLUX, LIM>(&sW[0][tj][ti], TR, a.gam, a.igm1, f, VS);
#pragma unroll
        for (int v = 0; v < NV; ++v) sFt[v][tj][ti] = f[v];
      }
      for (int q = tid - 64; q >= 0 && q < TR; q += NT - 64) {
        if (q >= 2 && q < TR - 2) {
          R f[NV];
          lds_face<R, 2, FLUX, LIM>(&sW[0][TT][q], TR, a.gam, a.igm1, f, VS);
#pragma unroll
          for (int v = 0; v < NV; ++v) sFt[v][TT][q] = f[v];
        }
      }
    }
    // Stage 2: the own cell's U^n for the RK combine is loaded here, before
    // the phi face and the barrier, so that its latency overlaps that work
    // instead of stalling the update.
    R up[NV];
    if (STAGE == 2 && body && valid) {
      const unsigned c = kbase + colbase;
#pragma unroll
      for (int v = 0; v < NV; ++v) up[v] = ldg(a.un + v * a.ncell, c);
    }
    // phi face k+1/2 from the register ring (and the next plane's load)
    R fhi[NV];
    {
      R wd[NV], wl[NV], wr[NV];
      own_cvt(uring, wd);      // W(k + 2), loaded one plane ago
      own_raw(k + 3, uring);   // in flight until the next plane's phi face
      reconstruct<R, LIM, true>(wa, wb, wc, wd, wl, wr);
      face_flux<R, 3, FLUX, true>(wl, wr, a.gam, a.igm1, fhi);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        wa[v] = wb[v];
        wb[v] = wc[v];
        wc[v] = wd[v];
      }
    }
    // now wa = W(k), wb = W(k+1), wc = W(k+2)
    if (body) {
      __syncthreads();  // r / theta face fluxes are in LDS
      if constexpr (DMA) {
        if (dma_on && k + 1 < kend) dma_halo(k + 1);  // in flight during this update
      }
      if (valid) {
        const R rm2 = cm.r(MR_RM2), rp2 = cm.r(MR_RP2), ivr = cm.r(MR_IVR);
        const R hr = cm.r(MR_HR);
        const R sm = cm.t(MT_SM), sp = cm.t(MT_SP), ict = cm.t(MT_ICT);
        const R fph = hr * cm.t(MT_PHF);
        R L[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          L[v] = R(0);
          L[v] -= (rp2 * sFr[v][tj][ti + 1] - rm2 * sFr[v][tj][ti]) * ivr;
          L[v] -= hr * (sp * sFt[v][tj + 1][ti] - sm * sFt[v][tj][ti]) * ict;
          L[v] -= fph * (fhi[v] - fcar[v]);
        }
        add_sources_cm<R>(wa, cm, a.omega, a.gravity, a.corot, L);
        // the stage's own conserved state, rebuilt from the ring's primitives
        // (equal to the stored values up to rounding; no reload)
        R uc[NV];
        prim2cons<R>(wa, uc, a.igm1);
        const unsigned c = kbase + colbase;
        if constexpr (FM) {  // passive tracer on: keep this stage's mass fluxes
          stg(a.fmass, c, sFr[0][tj][ti]);
          stg(a.fmass + a.ncell, c, sFt[0][tj][ti]);
          stg(a.fmass + 2 * a.ncell, c, fcar[0]);
          if (i == nr - 1) stg(a.fmass_rout, (unsigned)(k * nt + j), sFr[0][tj][ti + 1]);
          if (j == nt - 1) stg(a.fmass_tend, (unsigned)(k * nr + i), sFt[0][tj + 1][ti]);
        }
        if (STAGE == 1) {
#pragma unroll
          for (int v = 0; v < NV; ++v) stg(a.uout + v * a.ncell, c, uc[v] + dt * L[v]);
        } else {
          R un[NV], unew[NV], wn[NV];
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            un[v] = up[v];
            unew[v] = R(0.5) * un[v] + R(0.5) * (uc[v] + dt * L[v]);
            stg(a.uout + v * a.ncell, c, unew[v]);
          }
          cons2prim<R, true>(unew, wn, a.gm1);
          lam = fmax(lam, cell_rate_cm<R, true>(wn, cm, a.gam));
          const double d = (double)unew[0] - (double)un[0];
          s1 += d * d;
          s0 += (double)un[0] * (double)un[0];
          if (bad == BAD_NONE && !cell_valid<R>(unew, wn)) bad = (int)c;
        }
      }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) fcar[v] = fhi[v];
  }
  if (STAGE == 2) write_partials(a.partials, pslot, lam, s1, s0, bad);
}


// ------------------------------------------------------------ finalize --
// Reduce the stage-2 (or CFL) block partials in a fixed order, advance the
// clock, set the next dt; then, if probes are logged, append a record.
template <typename R>
__device__ __forceinline__ void finalize_run(DevClock* ck, const double* __restrict__ part,
                                             int nblocks, double cfl, int advance, int log_on,
                                             const ProbeArgs& pa, const R* __restrict__ u,
                                             double* __restrict__ log) {
  __shared__ double sh[4][4];
  __shared__ int s_rec;
  __shared__ long long s_row, s_idx;
  __shared__ double s_t;
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  const int nthr = blockDim.x * blockDim.y;
  if (!ck->active && advance) return;  // the stage kernels did not run
  double l = 0.0, a1 = 0.0, a0 = 0.0;
  int b = BAD_NONE;
  for (int q = tid; q < nblocks; q += nthr) {
    l = fmax(l, part[4 * q + 0]);
    a1 += part[4 * q + 1];
    a0 += part[4 * q + 2];
    const int qb = (int)part[4 * q + 3];
    b = qb < b ? qb : b;
  }
  block_reduce(l, a1, a0, b, sh);
  if (tid == 0) {
    if (advance) {
      ck->t = ck->clip ? ck->t_end : ck->t + ck->dt;
      ck->step += 1;
      ck->taken += 1;
      ck->last_dt = ck->dt;
      ck->resid = sqrt(a1) / sqrt(a0);
      if (b != BAD_NONE) {
        if (ck->bad == BAD_NONE || b < ck->bad) ck->bad = b;
      }
    }
    set_next_dt(ck, cfl / l);
    if (ck->bad != BAD_NONE) ck->active = 0;
    // probe cadence decision on the new time
    int rec = advance;
    long long idx = 0;
    if (rec && pa.cadence > 0.0) {
      idx = (long long)floor(ck->t * pa.sc.t / pa.cadence);
      rec = idx > ck->last_sample;
    }
    s_rec = log_on && rec;
    s_row = ck->n_log;
    s_idx = idx;
    s_t = ck->t;
    if (log_on && rec) {
      ck->n_log += 1;
      if (pa.cadence > 0.0) ck->last_sample = idx;
    }
  }
  __syncthreads();
  if (s_rec && s_row < pa.log_rows && tid < pa.n)
    probe_eval<R>(pa, u, tid, s_t, log + (s_row * pa.max_probes + tid) * 12);
}


}  // namespace icr
