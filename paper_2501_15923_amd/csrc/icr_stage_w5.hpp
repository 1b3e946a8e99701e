// icr_stage_w5.hpp -- face-once stage tile for the WENO5 reconstruction
// (three ghost layers, six-cell stencils), the counterpart of stage_tile in
// icr_stage_lds.hpp for the minmod / MC limiters.
//
// A block of 64 x 4 threads marches along phi over a chunk of planes; each
// row of 64 lanes covers 58 cells plus the three-cell r halo on either side.
// Per plane the primitives of the tile's rows plus a three-row theta halo
// sit in LDS; every face flux is computed once and shared by its two cells.
// In every direction each cell forms both of its WENO5 edge values from its
// five-cell stencil (the two mirrored reconstructions share the smoothness
// indicators), and a face pairs the upper value of the cell below with the
// lower value of the cell above: along r the lane below is one lane down in
// the same wave (a wave is one row), along theta the row below is another
// wave and its values pass through LDS, along phi the previous plane's
// value is carried in registers.  Each thread keeps the primitives of
// planes k-1 .. k+2 of its own column (and loads k+3), the upper phi edge
// value of cell k and the flux of face k-1/2 from the previous plane.
// WENO5 works on primitive variables like the slope
// limiters (Jiang & Shu 1996 weights, a face state with rho or p <= 0 falls
// back to its cell value); the weight normalisation multiplies by the
// Newton-refined reciprocal, as the fluxes do.  Stage 2 also forms the
// per-block partials of the next CFL dt, of the relaxation residual and of
// the validity flag.
#pragma once
#include "icr_stage_lds.hpp"

namespace icr {

constexpr int W5_TR = 64, W5_TT = 4, W5_H = 3;
constexpr int W5_TI = W5_TR - 2 * W5_H;  // cells along r per tile row

// Both WENO5 edge values of the cell c from the five cells a..e: up = the
// value at the face between c and d (weno5(a, b, c, d, e)), dn = the value
// at the face between b and c (weno5(e, d, c, b, a)).  The mirrored stencil
// has the same three smoothness indicators in reverse order and the same
// eps, so they are formed once; the expressions are symmetric under
// a..e -> e..a, so a mirror-symmetric flow keeps mirror-symmetric states.
// Equal to the two weno5 calls up to rounding.
template <typename R, bool FAST = false>
__device__ __forceinline__ void weno5_cell(R a, R b, R c, R d, R e, R& up, R& dn) {
  const R s0 = (a + c) - R(2) * b, t0 = (a - R(4) * b) + R(3) * c;
  const R s1 = (b + d) - R(2) * c, t1 = b - d;
  const R s2 = (e + c) - R(2) * d, t2 = (e - R(4) * d) + R(3) * c;
  const R b0 = R(13) / R(12) * s0 * s0 + R(0.25) * t0 * t0;
  const R b1 = R(13) / R(12) * s1 * s1 + R(0.25) * t1 * t1;
  const R b2 = R(13) / R(12) * s2 * s2 + R(0.25) * t2 * t2;
  const R eps = R(1e-6) * ((a * a + e * e) + (b * b + d * d) + c * c) * R(0.2) +
                (sizeof(R) == 8 ? R(1e-40) : R(1e-15));
  const R g0 = (eps + b0) * (eps + b0), g1 = (eps + b1) * (eps + b1), g2 = (eps + b2) * (eps + b2);
  // candidates times 6: up uses the stencils ending at / centred on /
  // starting at c read from a, dn the same read from e
  const R u0 = (R(2) * a - R(7) * b) + R(11) * c, u1 = (R(5) * c - b) + R(2) * d;
  const R u2 = (R(2) * c - e) + R(5) * d;
  const R d0 = (R(2) * e - R(7) * d) + R(11) * c, d1 = (R(5) * c - d) + R(2) * b;
  const R d2 = (R(2) * c - a) + R(5) * b;
  constexpr R sixth = R(1) / R(6);
  if constexpr (sizeof(R) == 8) {
    // weights d_k / g_k scaled by g0 g1 g2 (one reciprocal per value)
    const R p12 = g1 * g2, p02 = g0 * g2, p01 = g0 * g1;
    const R ua0 = R(0.1) * p12, ua1 = R(0.6) * p02, ua2 = R(0.3) * p01;
    const R da0 = R(0.1) * p01, da2 = R(0.3) * p12;
    const R un = ua0 * u0 + ua1 * u1 + ua2 * u2, us = ua0 + ua1 + ua2;
    const R dnn = da0 * d0 + ua1 * d1 + da2 * d2, ds = da0 + ua1 + da2;
    if constexpr (FAST) {
      up = un * rcp_fast(us) * sixth;
      dn = dnn * rcp_fast(ds) * sixth;
    } else {
      up = un / us * sixth;
      dn = dnn / ds * sixth;
    }
  } else {
    const R i0 = FAST ? rcp_fast(g0) : R(1) / g0;
    const R i1 = FAST ? rcp_fast(g1) : R(1) / g1;
    const R i2 = FAST ? rcp_fast(g2) : R(1) / g2;
    const R ua0 = R(0.1) * i0, ua1 = R(0.6) * i1, ua2 = R(0.3) * i2;
    const R da0 = R(0.1) * i2, da2 = R(0.3) * i0;
    const R un = ua0 * u0 + ua1 * u1 + ua2 * u2, us = ua0 + ua1 + ua2;
    const R dnn = da0 * d0 + ua1 * d1 + da2 * d2, ds = da0 + ua1 + da2;
    up = un / us * sixth;
    dn = dnn / ds * sixth;
  }
}

// Both edge values of a variable are complete here: without this the
// compiler forms every variable's upper values first (the shuffle needs
// them) and keeps the inputs of all lower values live, which spills.  The
// empty asm emits no instruction.
template <typename R>
__device__ __forceinline__ void pin(R& x, R& y) {
  asm volatile("" : "+v"(x), "+v"(y));
}

template <typename R>
struct alignas(16) StageW5 {
  R sW[NV][W5_TT + 2 * W5_H][W5_TR];  // primitives, rows j0-3 .. j0+TT+2
  R sFr[NV][W5_TT][W5_TR];            // r face i-1/2 at the lane of cell i
  R sFt[NV][W5_TT + 1][W5_TR];        // theta face j-1/2 at row j (0 .. TT)
};

template <typename R, int FLUX, int STAGE>
__device__ __forceinline__ void stage_tile_w5(const StageArgs<R>& a, int kplanes, int bx, int by,
                                              int bz, int pslot, StageW5<R>& sm) {
  constexpr int TR = W5_TR, TT = W5_TT, H = W5_H, NT = TR * TT, WT = TT + 2 * H;
  auto& sW = sm.sW;
  auto& sFr = sm.sFr;
  auto& sFt = sm.sFt;

  const int ti = threadIdx.x, tj = threadIdx.y, tid = tj * TR + ti;
  const int i0 = bx * W5_TI, j0 = by * TT, k0 = bz * kplanes;
  const int nr = a.nr, nt = a.nt, np = a.np;
  const int kend = k0 + kplanes < np ? k0 + kplanes : np;
  const int i = i0 + ti - H, j = j0 + tj;  // this lane's cell
  const bool inner = ti >= H && ti < TR - H;
  const bool valid = inner && i < nr && j < nt;
  // own column: the cell itself, the last cell beyond r_out; below r_in
  // cell 0, or under the asymm rule the mirror cell -1 - i
  const int ic = i < 0 ? (a.asymm ? (-1 - i < nr ? -1 - i : nr - 1) : 0)
                       : (i < nr ? i : nr - 1);
  const int jc = j < nt ? j : nt - 1;
  const unsigned colbase = (unsigned)(jc * nr + ic);
  bool flipj;
  const int mj = mirror_row(j, nt, flipj);
  const unsigned lbase = (unsigned)(mj * nr + ic);
  const bool lghost = i < 0;
  const unsigned plane_cells = (unsigned)(nt * nr);
  const long long gplane = (long long)nt * np;
  auto load_own = [&](int k, R (&w)[NV]) {
    load_cons_prim<R, true>(a, (unsigned)wrap_phi(k, np) * plane_cells + lbase, w);
    if (flipj) flip_theta(w);
  };

  if (!a.clock->active) {
    if (STAGE == 2 && valid)
      for (int k = k0; k < kend; ++k) {
        const unsigned c = (unsigned)k * plane_cells + colbase;
#pragma unroll
        for (int v = 0; v < NV; ++v) stg(a.uout + v * a.ncell, c, ldg(a.un + v * a.ncell, c));
      }
    return;
  }
  const R dt = (R)a.clock->dt;

  // phi ring: at the top of iteration k, w0 .. w3 = W(k-1) .. W(k+2),
  // ecar = the upper phi edge value of cell k (face k+1/2, left state) and
  // fcar = flux of face k-1/2; iteration k0-2 only forms ecar, k0-1 only
  // ecar and fcar
  R w0[NV], w1[NV], w2[NV], w3[NV], ecar[NV], fcar[NV];
  load_own(k0 - 3, w0);
  load_own(k0 - 2, w1);
  load_own(k0 - 1, w2);
  load_own(k0, w3);
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    fcar[v] = R(0);
    ecar[v] = R(0);
  }

  // r edge lane: lane l reads lanes l-2 .. l+2; lanes 2 .. TR-3 give the
  // edge values of the faces the update reads (lanes H .. TR-H); the outer
  // two lanes on either side repeat their neighbour's (never read)
  const int tc = ti < 2 ? 2 : (ti > TR - 3 ? TR - 3 : ti);

  double lam = 0.0, s1 = 0.0, s0 = 0.0;
  int bad = BAD_NONE;

  for (int k = k0 - 2; k < kend; ++k) {
    const bool body = k >= k0;  // uniform over the block
    const unsigned kbase = (unsigned)k * plane_cells;
    if (body) {
      __syncthreads();  // the previous plane's LDS reads are complete
      if (lghost) {  // inner ghost (primitives), the same in every layer
        R w[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) w[v] = ldg(a.ghost + v * gplane, (unsigned)(k * nt + mj));
        if (flipj) flip_theta(w);
        if (a.asymm) {  // w1: the mirror cell's primitives (already flipped)
          w[2] = -w1[2];
          w[3] = -w1[3];
          w[6] = -w1[6];
          w[7] = -w1[7];
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) sW[v][tj + H][ti] = w[v];
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) sW[v][tj + H][ti] = w1[v];
      }
      // theta halo: rows -3 .. -1 and TT .. TT+2 over all TR lanes
      for (int h = tid; h < 2 * H * TR; h += NT) {
        const int row = h / TR, l = h - row * TR;
        const int jj = row < H ? row - H : TT + row - H;
        const int gi = i0 + l - H;
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
        for (int v = 0; v < NV; ++v) sW[v][jj + H][l] = w[v];
      }
      __syncthreads();
      constexpr int VS = WT * TR;
      {
        // both r edge values of the lane's cell from lanes tc-2 .. tc+2; the
        // face i-1/2 takes the upper value of lane ti-1 (one lane up in the
        // wave, the row being one wave) and the lower value of lane ti
        R eu[NV], ed[NV], f[NV];
        const R* q = &sW[0][tj + H][tc];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          weno5_cell<R, true>(q[v * VS - 2], q[v * VS - 1], q[v * VS], q[v * VS + 1],
                              q[v * VS + 2], eu[v], ed[v]);
          pin(eu[v], ed[v]);
        }
        if (!(eu[0] > R(0) && eu[4] > R(0)))
#pragma unroll
          for (int v = 0; v < NV; ++v) eu[v] = q[v * VS];
        if (!(ed[0] > R(0) && ed[4] > R(0)))
#pragma unroll
          for (int v = 0; v < NV; ++v) ed[v] = q[v * VS];
#pragma unroll
        for (int v = 0; v < NV; ++v) eu[v] = __shfl_up(eu[v], 1, 64);
        face_flux<R, 1, FLUX, true>(eu, ed, a.gam, a.igm1, f);
#pragma unroll
        for (int v = 0; v < NV; ++v) sFr[v][tj][ti] = f[v];
      }
      // theta: both edge values of the lane's cell from sW rows tj+1 ..
      // tj+5; wave 0 also forms the upper value of the row below the tile
      // (cell j0-1) and wave TT-1 the lower value of the row above it (cell
      // j0+TT), with the same expressions as the neighbouring tiles, so a
      // face shared by two tiles gets the same flux in both
      R tu[NV], td[NV], xe[NV];
      {
        const R* q = &sW[0][tj + H][ti];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          weno5_cell<R, true>(q[v * VS - 2 * TR], q[v * VS - TR], q[v * VS], q[v * VS + TR],
                              q[v * VS + 2 * TR], tu[v], td[v]);
          pin(tu[v], td[v]);
        }
        if (!(tu[0] > R(0) && tu[4] > R(0)))
#pragma unroll
          for (int v = 0; v < NV; ++v) tu[v] = q[v * VS];
        if (!(td[0] > R(0) && td[4] > R(0)))
#pragma unroll
          for (int v = 0; v < NV; ++v) td[v] = q[v * VS];
      }
      const bool lo_wave = tj == 0, hi_wave = tj == TT - 1;  // uniform per wave
      if (lo_wave || hi_wave) {
        const R* q = &sW[0][lo_wave ? H - 1 : TT + H][ti];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          R eu, ed;
          weno5_cell<R, true>(q[v * VS - 2 * TR], q[v * VS - TR], q[v * VS], q[v * VS + TR],
                              q[v * VS + 2 * TR], eu, ed);
          xe[v] = lo_wave ? eu : ed;
        }
        if (!(xe[0] > R(0) && xe[4] > R(0)))
#pragma unroll
          for (int v = 0; v < NV; ++v) xe[v] = q[v * VS];
      }
      // the left states of the faces at rows 0 .. TT-1 go through the flux
      // rows (row tj is then read and overwritten by wave tj alone): the
      // upper values of rows 0 .. TT-2 and of the row below the tile; wave
      // TT-1 finishes the tile's upper face (row TT) from its own values
      if (!hi_wave)
#pragma unroll
        for (int v = 0; v < NV; ++v) sFt[v][tj + 1][ti] = tu[v];
      if (lo_wave)
#pragma unroll
        for (int v = 0; v < NV; ++v) sFt[v][0][ti] = xe[v];
      if (hi_wave) {
        R f[NV];
        face_flux<R, 2, FLUX, true>(tu, xe, a.gam, a.igm1, f);
#pragma unroll
        for (int v = 0; v < NV; ++v) sFt[v][TT][ti] = f[v];
      }
      __syncthreads();
      {
        R lft[NV], f[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) lft[v] = sFt[v][tj][ti];
        face_flux<R, 2, FLUX, true>(lft, td, a.gam, a.igm1, f);
#pragma unroll
        for (int v = 0; v < NV; ++v) sFt[v][tj][ti] = f[v];
      }
    }
    // stage 2: the own cell's U^n for the RK combine, issued early
    R up[NV];
    if (STAGE == 2 && body && valid) {
      const unsigned c = kbase + colbase;
#pragma unroll
      for (int v = 0; v < NV; ++v) up[v] = ldg(a.un + v * a.ncell, c);
    }
    // phi edge values of cell k+1 from W(k-1) .. W(k+3); face k+1/2 from
    // the carried upper value of cell k and the lower value of cell k+1
    R fhi[NV];
    {
      R w4[NV], eu[NV], ed[NV];
      load_own(k + 3, w4);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        weno5_cell<R, true>(w0[v], w1[v], w2[v], w3[v], w4[v], eu[v], ed[v]);
        pin(eu[v], ed[v]);
      }
      if (!(eu[0] > R(0) && eu[4] > R(0)))
#pragma unroll
        for (int v = 0; v < NV; ++v) eu[v] = w2[v];
      if (!(ed[0] > R(0) && ed[4] > R(0)))
#pragma unroll
        for (int v = 0; v < NV; ++v) ed[v] = w2[v];
      if (k >= k0 - 1)
        face_flux<R, 3, FLUX, true>(ecar, ed, a.gam, a.igm1, fhi);
      else
#pragma unroll
        for (int v = 0; v < NV; ++v) fhi[v] = R(0);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        ecar[v] = eu[v];
        w0[v] = w1[v];
        w1[v] = w2[v];
        w2[v] = w3[v];
        w3[v] = w4[v];
      }
    }
    // now w0 = W(k), w1 = W(k+1)
    if (body) {
      __syncthreads();  // r / theta face fluxes are in LDS
      if (valid) {
        const R rm2 = ldg(a.m.rm2, ic), rp2 = ldg(a.m.rp2, ic), ivr = ldg(a.m.ivr, ic);
        const R hr = ldg(a.m.hr, ic);
        const R sm = ldg(a.m.sm, jc), sp = ldg(a.m.sp, jc), ict = ldg(a.m.ict, jc);
        const R fph = hr * ldg(a.m.phf, jc);
        R L[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          L[v] = R(0);
          L[v] -= (rp2 * sFr[v][tj][ti + 1] - rm2 * sFr[v][tj][ti]) * ivr;
          L[v] -= hr * (sp * sFt[v][tj + 1][ti] - sm * sFt[v][tj][ti]) * ict;
          L[v] -= fph * (fhi[v] - fcar[v]);
        }
        add_sources<R>(w0, a.m, ic, jc, a.omega, a.gravity, a.corot, L);
        R uc[NV];
        prim2cons<R>(w0, uc, a.igm1);
        const unsigned c = kbase + colbase;
        if (STAGE == 1) {
#pragma unroll
          for (int v = 0; v < NV; ++v) stg(a.uout + v * a.ncell, c, uc[v] + dt * L[v]);
        } else {
          R unew[NV], wn[NV];
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            unew[v] = R(0.5) * up[v] + R(0.5) * (uc[v] + dt * L[v]);
            stg(a.uout + v * a.ncell, c, unew[v]);
          }
          cons2prim<R, true>(unew, wn, a.gm1);
          lam = fmax(lam, cell_rate<R, true>(wn, a.m, ic, jc, a.gam));
          const double d = (double)unew[0] - (double)up[0];
          s1 += d * d;
          s0 += (double)up[0] * (double)up[0];
          if (bad == BAD_NONE && !cell_valid<R>(unew, wn)) bad = (int)c;
        }
      }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) fcar[v] = fhi[v];
  }
  if (STAGE == 2) write_partials(a.partials, pslot, lam, s1, s0, bad);
}

}  // namespace icr
