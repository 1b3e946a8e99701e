// icr_stage_w5.hpp -- face-once stage tile for the WENO5 reconstruction
// (three ghost layers, six-cell stencils), the counterpart of stage_tile in
// icr_stage_lds.hpp for the minmod / MC limiters.
//
// A block of 64 x 4 threads marches along phi over a chunk of planes; each
// row of 64 lanes covers 58 cells plus the three-cell r halo on either side.
// Per plane the primitives of the tile's rows plus a three-row theta halo
// sit in LDS; every r and theta face flux is computed once, from six LDS
// values per variable, and shared by its two cells.  The phi direction is
// carried in registers: each thread keeps the primitives of planes k-2 ..
// k+2 of its own column (and loads k+3) and the flux of face k-1/2 from the
// previous plane.  WENO5 works on primitive variables like the slope
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

template <typename R>
struct alignas(16) StageW5 {
  R sW[NV][W5_TT + 2 * W5_H][W5_TR];  // primitives, rows j0-3 .. j0+TT+2
  R sFr[NV][W5_TT][W5_TR];            // r face i-1/2 at the lane of cell i
  R sFt[NV][W5_TT + 1][W5_TR];        // theta face j-1/2 at row j (0 .. TT)
};

// Face m-1/2 from the six LDS values of cells m-3 .. m+2 (stride apart) of
// every variable (vstride apart), then the numerical flux.  One variable at
// a time keeps six values live; the cell-value fallback rereads LDS.
template <typename R, int N, int FLUX>
__device__ __forceinline__ void lds_face_w5(const R* base, int stride, int vstride, R gam,
                                            R igm1, R (&f)[NV]) {
  R wl[NV], wr[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const R* q = base + v * vstride;
    const R p0 = q[0], p1 = q[stride], p2 = q[2 * stride], p3 = q[3 * stride];
    const R p4 = q[4 * stride], p5 = q[5 * stride];
    wl[v] = weno5<R, true>(p0, p1, p2, p3, p4);
    wr[v] = weno5<R, true>(p5, p4, p3, p2, p1);
  }
  if (!(wl[0] > R(0) && wl[4] > R(0)))
#pragma unroll
    for (int v = 0; v < NV; ++v) wl[v] = base[v * vstride + 2 * stride];
  if (!(wr[0] > R(0) && wr[4] > R(0)))
#pragma unroll
    for (int v = 0; v < NV; ++v) wr[v] = base[v * vstride + 3 * stride];
  face_flux<R, N, FLUX, true>(wl, wr, gam, igm1, f);
}

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

  // phi ring: at the top of iteration k, w0 .. w4 = W(k-2) .. W(k+2) and
  // fcar = flux of face k-1/2; iteration k0-1 only forms fcar
  R w0[NV], w1[NV], w2[NV], w3[NV], w4[NV], fcar[NV];
  load_own(k0 - 3, w0);
  load_own(k0 - 2, w1);
  load_own(k0 - 1, w2);
  load_own(k0, w3);
  load_own(k0 + 1, w4);
#pragma unroll
  for (int v = 0; v < NV; ++v) fcar[v] = R(0);

  // r face lane: the stencil of lane l reads lanes l-3 .. l+2; halo lanes
  // take the nearest interior lane's face (never read by the update)
  const int tf = ti < H ? H : (ti > TR - H ? TR - H : ti);

  double lam = 0.0, s1 = 0.0, s0 = 0.0;
  int bad = BAD_NONE;

  for (int k = k0 - 1; k < kend; ++k) {
    const bool body = k >= k0;  // uniform over the block
    const unsigned kbase = (unsigned)k * plane_cells;
    if (body) {
      __syncthreads();  // the previous plane's LDS reads are complete
      if (lghost) {  // inner ghost (primitives), the same in every layer
        R w[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) w[v] = ldg(a.ghost + v * gplane, (unsigned)(k * nt + mj));
        if (flipj) flip_theta(w);
        if (a.asymm) {  // w2: the mirror cell's primitives (already flipped)
          w[2] = -w2[2];
          w[3] = -w2[3];
          w[6] = -w2[6];
          w[7] = -w2[7];
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) sW[v][tj + H][ti] = w[v];
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) sW[v][tj + H][ti] = w2[v];
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
        R f[NV];
        lds_face_w5<R, 1, FLUX>(&sW[0][tj + H][tf] - H, 1, VS, a.gam, a.igm1, f);
#pragma unroll
        for (int v = 0; v < NV; ++v) sFr[v][tj][ti] = f[v];
      }
      {
        R f[NV];
        lds_face_w5<R, 2, FLUX>(&sW[0][tj][ti], TR, VS, a.gam, a.igm1, f);
#pragma unroll
        for (int v = 0; v < NV; ++v) sFt[v][tj][ti] = f[v];
      }
      // the tile's upper theta face (row TT) of the inner lanes: wave 1
      for (int q = tid - 64; q >= 0 && q < TR; q += NT - 64) {
        if (q >= H && q < TR - H) {
          R f[NV];
          lds_face_w5<R, 2, FLUX>(&sW[0][TT][q], TR, VS, a.gam, a.igm1, f);
#pragma unroll
          for (int v = 0; v < NV; ++v) sFt[v][TT][q] = f[v];
        }
      }
    }
    // stage 2: the own cell's U^n for the RK combine, issued early
    R up[NV];
    if (STAGE == 2 && body && valid) {
      const unsigned c = kbase + colbase;
#pragma unroll
      for (int v = 0; v < NV; ++v) up[v] = ldg(a.un + v * a.ncell, c);
    }
    // phi face k+1/2 from W(k-2) .. W(k+3)
    R fhi[NV];
    {
      R w5[NV], wl[NV], wr[NV];
      load_own(k + 3, w5);
      reconstruct_weno5<R, true>(w0, w1, w2, w3, w4, w5, wl, wr);
      face_flux<R, 3, FLUX, true>(wl, wr, a.gam, a.igm1, fhi);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        w0[v] = w1[v];
        w1[v] = w2[v];
        w2[v] = w3[v];
        w3[v] = w4[v];
        w4[v] = w5[v];
      }
    }
    // now w1 = W(k), w2 = W(k+1)
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
        add_sources<R>(w1, a.m, ic, jc, a.omega, a.gravity, a.corot, L);
        R uc[NV];
        prim2cons<R>(w1, uc, a.igm1);
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
