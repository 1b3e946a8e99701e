// icr_amr.hip -- block-structured adaptive mesh refinement of the
// heliospheric update (the refined runs of Sect. 3.2 and Sect. 4: blocks
// refined where the CME tracer or a compression is present, criteria
// 'tracing', 'shock', 'combined').
//
// Blocks of br x bt x bp cells at every level, each held with two ghost
// layers; a level-(l+1) block is one octant of a level-l block at twice the
// resolution (radial edges split at the geometric mean).  One global dt,
// SSP-RK2 on the leaves.  Per stage:
//   k_amr_ghost   the ghost layers of every leaf, coarse levels first: copies
//                 from a leaf of the same level, volume-weighted restriction
//                 of finer leaves, conservative prolongation of the coarser
//                 leaf (minmod slopes from its padded block, then a constant
//                 correction so the children's volume-weighted mean is the
//                 coarse cell), physical edges as in the uniform solver;
//   k_amr_stage   reconstruct / flux / divergence / sources / RK combine of
//                 every leaf cell, the fluxes of the block's six faces kept;
//   k_amr_reflux  a coarse cell next to finer leaves takes the area-weighted
//                 sum of their face fluxes instead of its own on that face.
// After a step: the CFL rate of every leaf cell (one-block finalize), and
// every regrid_every steps the block indicators (max tau, max compression)
// that the host turns into splits (k_amr_prolong) and merges
// (k_amr_restrict), keeping face neighbours within one level.
// The passive CME tracer rho tau rides along as a ninth conserved variable.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <set>
#include <string>
#include <vector>

#include "icarus_hip.h"
#include "icr_kernels.hpp"

namespace icr {

int set_error(int code, const char* msg);  // icr_api.hip

constexpr int AMR_MAXL = 6;
constexpr int NA = 9;   // conserved variables + rho tau
constexpr int AG = 2;   // ghost layers

struct AmrLevel {
  Metric<double> m;
  const double* m64;  // edges and colatitude centres (k_metric layout)
  const int* map;     // [nbp][nbt][nbr] -> block slot, -1 where no block
  int nr, nt, np, nbr, nbt, nbp;
  double dth, dph;
};

struct AmrArgs {
  double* U;   // [slot][9][pp][pt][pr] U^n / U^{n+1}
  double* U1;  // [slot][9][pp][pt][pr] stage-1 state
  double* F;   // [slot][6][9][fmax] fluxes of the block faces r-, r+, t-, t+, p-, p+
  const unsigned char* leaf;  // [slot]
  const int* key;             // [slot][4]: level, bi, bj, bk
  AmrLevel lv[AMR_MAXL + 1];  // index = level (1 ..)
  int nlev, br, bt, bp, pr, pt, pp, fmax;
  long long bvol;  // padded cells per variable of a block
  BndArgs bnd;     // maps and CMEs on the base grid
  DevClock* clock;
  double* partials;
  double gam, gm1, igm1, omega, cfl, r_in;
  int gravity, corot;
};

__device__ __forceinline__ long long pidx(const AmrArgs& a, int slot, int v, int kk, int jj,
                                          int ii) {
  return (long long)slot * NA * a.bvol + ((long long)(v * a.pp + kk) * a.pt + jj) * a.pr + ii;
}

__device__ __forceinline__ int face_cells(const AmrArgs& a, int d) {
  return d == 0 ? a.bp * a.bt : (d == 1 ? a.bp * a.br : a.bt * a.br);
}

__device__ __forceinline__ long long fidx(const AmrArgs& a, int slot, int face, int v, int q) {
  return (((long long)slot * 6 + face) * NA + v) * a.fmax + q;
}

__device__ __forceinline__ int amr_slot(const AmrArgs& a, int l, int i, int j, int k) {
  const AmrLevel& L = a.lv[l];
  return L.map[((long long)(k / a.bp) * L.nbt + j / a.bt) * L.nbr + i / a.br];
}

// Cell volume without the phi width, and the full volume, at level l.
__device__ __forceinline__ double vol_nophi(const AmrArgs& a, int l, int i, int j) {
  const Metric<double>& m = a.lv[l].m;
  return 1.0 / (m.ivr[i] * m.ict[j]);
}

// Inner-boundary primitive of level-l column (j, k): the map of the base
// column containing it (time interpolated), the cone CME tested at this
// column's centre; *inside = 1 inside an inserted cone.
__device__ void amr_inner_prim(const AmrArgs& a, int l, int j, int k, double t, double (&w)[NV],
                               int* inside) {
  const int f = 1 << (l - 1);
  BndArgs maponly = a.bnd;  // the map of the base column; CMEs tested below
  maponly.n_cme = 0;
  boundary_prim(maponly, t, j / f, k / f, w, nullptr);
  *inside = 0;
  const double th = a.lv[l].m64[OFF_TC64(a.lv[l].nr, a.lv[l].nt) + j];
  const double ph = (k + 0.5) * a.lv[l].dph;
  const double sth = sin(th), cth = cos(th);
  for (int c = 0; c < a.bnd.n_cme; ++c) {
    const double* m = a.bnd.cme + 8 * c;
    if (!(t >= m[0] && t < m[0] + m[1])) continue;
    const double cosd = cth * cos(m[2]) + sth * sin(m[2]) * cos(ph - m[3]);
    if (cosd >= m[4]) {
      *inside = 1;
      w[0] = m[6];
      w[1] = m[5];
      w[2] = 0.0;
      w[3] = -a.omega * a.r_in * sth;
      w[4] = m[7];
    }
  }
}

__device__ __forceinline__ double mm(double x, double y) {
  return x * y <= 0.0 ? 0.0 : (fabs(x) < fabs(y) ? x : y);
}

// Children (sub = e*4 + b*2 + c for phi, theta, r halves) of a level-l
// coarse cell with centre value c0 and face neighbours n[6] (r-, r+, t-,
// t+, p-, p+), the cell at global (ic, jc): conservative prolongation of one
// variable; writes all 8 children.
__device__ void prolong8(const AmrArgs& a, int l, int ic, int jc, double c0,
                         const double (&n)[6], double (&ch)[8]) {
  const double sr = mm(c0 - n[0], n[1] - c0);
  const double st = mm(c0 - n[2], n[3] - c0);
  const double sp = mm(c0 - n[4], n[5] - c0);
  double vs = 0.0, ws = 0.0;
  for (int s = 0; s < 8; ++s) {
    const int e = s >> 2, b = (s >> 1) & 1, c = s & 1;
    const double x = c0 + sp * (e ? 0.25 : -0.25) + st * (b ? 0.25 : -0.25) +
                     sr * (c ? 0.25 : -0.25);
    ch[s] = x;
    const double v = vol_nophi(a, l + 1, 2 * ic + c, 2 * jc + b);
    vs += v;
    ws += x * v;
  }
  const double d = c0 - ws / vs;
  for (int s = 0; s < 8; ++s) ch[s] += d;
}

// The level-l cell (i, j, k) (inside the domain) of buffer `buf` from the
// leaves: a leaf of level l, the restriction of 8 finer leaf cells, or the
// prolongation of the coarser leaf's cell (from its padded block).
__device__ void amr_value(const AmrArgs& a, const double* buf, int l, int i, int j, int k,
                          double (&u)[NA]) {
  const int slot = amr_slot(a, l, i, j, k);
  if (slot >= 0 && a.leaf[slot]) {
    const int* key = a.key + 4 * slot;
    const int ii = AG + i - key[1] * a.br, jj = AG + j - key[2] * a.bt, kk = AG + k - key[3] * a.bp;
    for (int v = 0; v < NA; ++v) u[v] = buf[pidx(a, slot, v, kk, jj, ii)];
    return;
  }
  if (slot >= 0) {  // refined: volume-weighted mean of the 8 children
    if (l >= a.nlev) {  // cannot happen in a valid tree: poison, do not read
      for (int v = 0; v < NA; ++v) u[v] = __builtin_nan("");
      return;
    }
    double acc[NA], vs = 0.0;
    for (int v = 0; v < NA; ++v) acc[v] = 0.0;
    for (int s = 0; s < 8; ++s) {
      const int e = s >> 2, b = (s >> 1) & 1, c = s & 1;
      const int fi = 2 * i + c, fj = 2 * j + b, fk = 2 * k + e;
      const int fs = amr_slot(a, l + 1, fi, fj, fk);
      if (fs < 0) {  // cannot happen in a valid tree
        for (int v = 0; v < NA; ++v) u[v] = __builtin_nan("");
        return;
      }
      const int* key = a.key + 4 * fs;
      const int ii = AG + fi - key[1] * a.br, jj = AG + fj - key[2] * a.bt,
                kk = AG + fk - key[3] * a.bp;
      const double vol = vol_nophi(a, l + 1, fi, fj);
      vs += vol;
      for (int v = 0; v < NA; ++v) acc[v] += buf[pidx(a, fs, v, kk, jj, ii)] * vol;
    }
    for (int v = 0; v < NA; ++v) u[v] = acc[v] / vs;
    return;
  }
  // covered by the coarser leaf
  const int ic = i >> 1, jc = j >> 1, kc = k >> 1;
  const int cs = l > 1 ? amr_slot(a, l - 1, ic, jc, kc) : -1;
  if (cs < 0) {  // cannot happen in a valid tree (levels differ by one)
    for (int v = 0; v < NA; ++v) u[v] = __builtin_nan("");
    return;
  }
  const int* key = a.key + 4 * cs;
  const int ii = AG + ic - key[1] * a.br, jj = AG + jc - key[2] * a.bt, kk = AG + kc - key[3] * a.bp;
  const int sub = ((k - 2 * kc) << 2) | ((j - 2 * jc) << 1) | (i - 2 * ic);
  for (int v = 0; v < NA; ++v) {
    const double c0 = buf[pidx(a, cs, v, kk, jj, ii)];
    const double n[6] = {buf[pidx(a, cs, v, kk, jj, ii - 1)], buf[pidx(a, cs, v, kk, jj, ii + 1)],
                         buf[pidx(a, cs, v, kk, jj - 1, ii)], buf[pidx(a, cs, v, kk, jj + 1, ii)],
                         buf[pidx(a, cs, v, kk - 1, jj, ii)], buf[pidx(a, cs, v, kk + 1, jj, ii)]};
    double ch[8];
    prolong8(a, l - 1, ic, jc, c0, n, ch);
    u[v] = ch[sub];
  }
}

__device__ __forceinline__ void prim_to_cons9(const AmrArgs& a, const double (&w)[NV], double tr,
                                              double (&u)[NA]) {
  double c[NV];
  prim2cons<double>(w, c, a.igm1);
  for (int v = 0; v < NV; ++v) u[v] = c[v];
  u[8] = tr * w[0];
}

// ---------------------------------------------------------------- ghosts --
// One thread per ghost cell of the listed leaves of level l: r faces
// (2 sides x 2 layers x bp x bt), theta faces (2 x 2 x bp x br), phi faces
// (2 x 2 x bt x br).  Inside a step the fill follows the step clock (no work
// once t_end is reached); a regrid fills whatever the clock says (always).
__global__ void __launch_bounds__(256) k_amr_ghost(AmrArgs a, int l, const int* __restrict__ list,
                                                   int n, int use_u1, int t_plus_dt, int always) {
  const int nr_g = 4 * a.bp * a.bt, nt_g = 4 * a.bp * a.br, np_g = 4 * a.bt * a.br;
  const int per = nr_g + nt_g + np_g;
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (long long)per * n || !(always || a.clock->active)) return;
  const int slot = list[q / per];
  int r = (int)(q % per);
  double* buf = use_u1 ? a.U1 : a.U;
  const int* key = a.key + 4 * slot;
  const int i0 = key[1] * a.br, j0 = key[2] * a.bt, k0 = key[3] * a.bp;
  const AmrLevel& L = a.lv[l];
  int d, side, g, x, y;  // direction, side, layer 1..2, transverse indices
  if (r < nr_g) {
    d = 0;
  } else if (r < nr_g + nt_g) {
    d = 1;
    r -= nr_g;
  } else {
    d = 2;
    r -= nr_g + nt_g;
  }
  const int w2 = d == 0 ? a.bt : a.br;  // fastest transverse extent
  const int area = (d == 2 ? a.bt : a.bp) * w2;
  side = r / (2 * area);
  r -= side * 2 * area;
  g = r / area + 1;
  r -= (g - 1) * area;
  y = r / w2;  // slower transverse (phi for r/theta faces, theta for phi faces)
  x = r - y * w2;
  // padded and global indices of the ghost cell
  int ii, jj, kk;
  if (d == 0) {
    ii = side ? AG + a.br - 1 + g : AG - g;
    jj = AG + x;
    kk = AG + y;
  } else if (d == 1) {
    ii = AG + x;
    jj = side ? AG + a.bt - 1 + g : AG - g;
    kk = AG + y;
  } else {
    ii = AG + x;
    jj = AG + y;
    kk = side ? AG + a.bp - 1 + g : AG - g;
  }
  int i = i0 + ii - AG, j = j0 + jj - AG, k = k0 + kk - AG;
  double u[NA];
  if (d == 0 && i < 0) {  // inner boundary: the same value in both layers
    const double t = a.clock->t + (t_plus_dt ? a.clock->dt : 0.0);
    double w[NV];
    int inside;
    amr_inner_prim(a, l, j, k, t, w, &inside);
    prim_to_cons9(a, w, (double)inside, u);
  } else if (d == 0 && i >= L.nr) {  // zero gradient beyond r_out
    for (int v = 0; v < NA; ++v) u[v] = buf[pidx(a, slot, v, kk, jj, AG + a.br - 1)];
  } else if (d == 1 && (j < 0 || j >= L.nt)) {  // mirror rows at the colatitude edges
    const int src = side ? AG + a.bt - g : AG + g - 1;
    for (int v = 0; v < NA; ++v) u[v] = buf[pidx(a, slot, v, kk, src, ii)];
    u[2] = -u[2];
    u[6] = -u[6];
  } else {
    if (d == 2) k = (k + L.np) % L.np;
    amr_value(a, buf, l, i, j, k, u);
  }
  for (int v = 0; v < NA; ++v) buf[pidx(a, slot, v, kk, jj, ii)] = u[v];
}

// ----------------------------------------------------------------- stage --
template <int FLUX, int LIM>
__device__ void amr_face(const AmrArgs& a, const double* buf, int slot, int d, int kk, int jj,
                         int ii, double (&f)[NA]) {
  // face between padded cells (kk, jj, ii) - e_d and (kk, jj, ii): cells
  // -2 .. +1 along d
  const int di = d == 0, dj = d == 1, dk = d == 2;
  double w[4][NV], rho[4], tr[4];
  for (int s = 0; s < 4; ++s) {
    const int o = s - 2;
    double u[NV];
    for (int v = 0; v < NV; ++v)
      u[v] = buf[pidx(a, slot, v, kk + o * dk, jj + o * dj, ii + o * di)];
    cons2prim<double>(u, w[s], a.gm1);
    rho[s] = u[0];
    tr[s] = buf[pidx(a, slot, 8, kk + o * dk, jj + o * dj, ii + o * di)];
  }
  double wl[NV], wr[NV], fl[NV];
  reconstruct<double, LIM>(w[0], w[1], w[2], w[3], wl, wr);
  if (d == 0)
    face_flux<double, 1, FLUX>(wl, wr, a.gam, a.igm1, fl);
  else if (d == 1)
    face_flux<double, 2, FLUX>(wl, wr, a.gam, a.igm1, fl);
  else
    face_flux<double, 3, FLUX>(wl, wr, a.gam, a.igm1, fl);
  for (int v = 0; v < NV; ++v) f[v] = fl[v];
  // tracer: mass flux times tau of the upwind cell
  f[8] = fl[0] * (fl[0] >= 0.0 ? tr[1] / rho[1] : tr[2] / rho[2]);
}

// One thread per cell of the listed leaves (blocks of 256 threads loop over
// a leaf's cells).  stage 1: U1 = U + dt L(U); stage 2: U = U/2 + (U1 + dt
// L(U1))/2 in place.
template <int FLUX, int LIM>
__global__ void __launch_bounds__(256) k_amr_stage(AmrArgs a, const int* __restrict__ list,
                                                   int stage) {
  if (!a.clock->active) return;
  const int slot = list[blockIdx.x];
  const int* key = a.key + 4 * slot;
  const int l = key[0];
  const AmrLevel& LV = a.lv[l];
  const Metric<double>& m = LV.m;
  const double dt = a.clock->dt;
  const double* in = stage == 1 ? a.U : a.U1;
  double* out = stage == 1 ? a.U1 : a.U;
  const int ncell = a.br * a.bt * a.bp;
  for (int c = threadIdx.x; c < ncell; c += blockDim.x) {
    const int ci = c % a.br, cj = (c / a.br) % a.bt, ck = c / (a.br * a.bt);
    const int ii = AG + ci, jj = AG + cj, kk = AG + ck;
    const int gi = key[1] * a.br + ci, gj = key[2] * a.bt + cj;
    double L[NA];
    for (int v = 0; v < NA; ++v) L[v] = 0.0;
    {  // r
      double fm[NA], fp[NA];
      amr_face<FLUX, LIM>(a, in, slot, 0, kk, jj, ii, fm);
      amr_face<FLUX, LIM>(a, in, slot, 0, kk, jj, ii + 1, fp);
      for (int v = 0; v < NA; ++v) L[v] -= (m.rp2[gi] * fp[v] - m.rm2[gi] * fm[v]) * m.ivr[gi];
      if (ci == 0)
        for (int v = 0; v < NA; ++v) a.F[fidx(a, slot, 0, v, ck * a.bt + cj)] = fm[v];
      if (ci == a.br - 1)
        for (int v = 0; v < NA; ++v) a.F[fidx(a, slot, 1, v, ck * a.bt + cj)] = fp[v];
    }
    {  // theta
      double fm[NA], fp[NA];
      amr_face<FLUX, LIM>(a, in, slot, 1, kk, jj, ii, fm);
      amr_face<FLUX, LIM>(a, in, slot, 1, kk, jj + 1, ii, fp);
      for (int v = 0; v < NA; ++v)
        L[v] -= m.hr[gi] * (m.sp[gj] * fp[v] - m.sm[gj] * fm[v]) * m.ict[gj];
      if (cj == 0)
        for (int v = 0; v < NA; ++v) a.F[fidx(a, slot, 2, v, ck * a.br + ci)] = fm[v];
      if (cj == a.bt - 1)
        for (int v = 0; v < NA; ++v) a.F[fidx(a, slot, 3, v, ck * a.br + ci)] = fp[v];
    }
    {  // phi
      double fm[NA], fp[NA];
      amr_face<FLUX, LIM>(a, in, slot, 2, kk, jj, ii, fm);
      amr_face<FLUX, LIM>(a, in, slot, 2, kk + 1, jj, ii, fp);
      const double fph = m.hr[gi] * m.phf[gj];
      for (int v = 0; v < NA; ++v) L[v] -= fph * (fp[v] - fm[v]);
      if (ck == 0)
        for (int v = 0; v < NA; ++v) a.F[fidx(a, slot, 4, v, cj * a.br + ci)] = fm[v];
      if (ck == a.bp - 1)
        for (int v = 0; v < NA; ++v) a.F[fidx(a, slot, 5, v, cj * a.br + ci)] = fp[v];
    }
    double u[NV], w[NV];
    for (int v = 0; v < NV; ++v) u[v] = in[pidx(a, slot, v, kk, jj, ii)];
    cons2prim<double>(u, w, a.gm1);
    double Ls[NV];
    for (int v = 0; v < NV; ++v) Ls[v] = L[v];
    add_sources<double>(w, m, gi, gj, a.omega, a.gravity, a.corot, Ls);
    for (int v = 0; v < NV; ++v) L[v] = Ls[v];
    for (int v = 0; v < NA; ++v) {
      const long long o = pidx(a, slot, v, kk, jj, ii);
      const double uc = in[o];
      out[o] = stage == 1 ? uc + dt * L[v] : 0.5 * out[o] + 0.5 * (uc + dt * L[v]);
    }
  }
}

// Face-once variant for leaves of at most 512 cells (two per thread): the
// faces of one direction at a time go to LDS (each computed once by
// amr_face, the same function and inputs as above, so the results are
// bitwise those of k_amr_stage), then every thread adds them to the
// right-hand sides of its cells, kept in registers.  Face index along
// direction d: position p in [0, b_d] (between cells p-1 and p) fastest for
// r, then the transverse cells.
constexpr int AMR_FO_CELLS = 512;
template <int FLUX, int LIM>
__global__ void __launch_bounds__(256) k_amr_stage_fo(AmrArgs a, const int* __restrict__ list,
                                                      int stage) {
  extern __shared__ double sF[];  // [NA][faces of one direction]
  if (!a.clock->active) return;
  const int slot = list[blockIdx.x];
  const int* key = a.key + 4 * slot;
  const int l = key[0];
  const AmrLevel& LV = a.lv[l];
  const Metric<double>& m = LV.m;
  const double dt = a.clock->dt;
  const double* in = stage == 1 ? a.U : a.U1;
  double* out = stage == 1 ? a.U1 : a.U;
  const int br = a.br, bt = a.bt, bp = a.bp;
  const int ncell = br * bt * bp;
  const int nfmax = (br + 1) * bt * bp > br * (bt + 1) * bp
                        ? ((br + 1) * bt * bp > br * bt * (bp + 1) ? (br + 1) * bt * bp
                                                                  : br * bt * (bp + 1))
                        : (br * (bt + 1) * bp > br * bt * (bp + 1) ? br * (bt + 1) * bp
                                                                  : br * bt * (bp + 1));
  double L[2][NA];
  for (int q = 0; q < 2; ++q)
    for (int v = 0; v < NA; ++v) L[q][v] = 0.0;
  for (int d = 0; d < 3; ++d) {
    const int nf = d == 0 ? (br + 1) * bt * bp : (d == 1 ? br * (bt + 1) * bp : br * bt * (bp + 1));
    for (int f = threadIdx.x; f < nf; f += blockDim.x) {
      int p, ci, cj, ck;  // face position along d and the transverse cells
      if (d == 0) {
        p = f % (br + 1);
        cj = (f / (br + 1)) % bt;
        ck = f / ((br + 1) * bt);
        ci = p;
      } else if (d == 1) {
        ci = f % br;
        p = (f / br) % (bt + 1);
        ck = f / (br * (bt + 1));
        cj = p;
      } else {
        ci = f % br;
        cj = (f / br) % bt;
        p = f / (br * bt);
        ck = p;
      }
      double fl[NA];
      amr_face<FLUX, LIM>(a, in, slot, d, AG + ck, AG + cj, AG + ci, fl);
      for (int v = 0; v < NA; ++v) sF[v * nfmax + f] = fl[v];
      const int bd = d == 0 ? br : (d == 1 ? bt : bp);
      if (p == 0 || p == bd) {  // block face: kept for the flux correction
        const int q = d == 0 ? ck * bt + cj : (d == 1 ? ck * br + ci : cj * br + ci);
        for (int v = 0; v < NA; ++v) a.F[fidx(a, slot, 2 * d + (p == bd), v, q)] = fl[v];
      }
    }
    __syncthreads();
    for (int q = 0; q < 2; ++q) {
      const int c = threadIdx.x + q * blockDim.x;
      if (c >= ncell) break;
      const int ci = c % br, cj = (c / br) % bt, ck = c / (br * bt);
      const int gi = key[1] * br + ci, gj = key[2] * bt + cj;
      if (d == 0) {
        const int f0 = (ck * bt + cj) * (br + 1) + ci;
        for (int v = 0; v < NA; ++v)
          L[q][v] -= (m.rp2[gi] * sF[v * nfmax + f0 + 1] - m.rm2[gi] * sF[v * nfmax + f0]) *
                     m.ivr[gi];
      } else if (d == 1) {
        const int f0 = (ck * (bt + 1) + cj) * br + ci;
        for (int v = 0; v < NA; ++v)
          L[q][v] -= m.hr[gi] *
                     (m.sp[gj] * sF[v * nfmax + f0 + br] - m.sm[gj] * sF[v * nfmax + f0]) *
                     m.ict[gj];
      } else {
        const int f0 = (ck * bt + cj) * br + ci;
        const double fph = m.hr[gi] * m.phf[gj];
        for (int v = 0; v < NA; ++v)
          L[q][v] -= fph * (sF[v * nfmax + f0 + br * bt] - sF[v * nfmax + f0]);
      }
    }
    __syncthreads();  // the next direction overwrites sF
  }
  for (int q = 0; q < 2; ++q) {
    const int c = threadIdx.x + q * blockDim.x;
    if (c >= ncell) break;
    const int ci = c % br, cj = (c / br) % bt, ck = c / (br * bt);
    const int ii = AG + ci, jj = AG + cj, kk = AG + ck;
    const int gi = key[1] * br + ci, gj = key[2] * bt + cj;
    double u[NV], w[NV];
    for (int v = 0; v < NV; ++v) u[v] = in[pidx(a, slot, v, kk, jj, ii)];
    cons2prim<double>(u, w, a.gm1);
    double Ls[NV];
    for (int v = 0; v < NV; ++v) Ls[v] = L[q][v];
    add_sources<double>(w, m, gi, gj, a.omega, a.gravity, a.corot, Ls);
    for (int v = 0; v < NV; ++v) L[q][v] = Ls[v];
    for (int v = 0; v < NA; ++v) {
      const long long o = pidx(a, slot, v, kk, jj, ii);
      const double uc = in[o];
      out[o] = stage == 1 ? uc + dt * L[q][v] : 0.5 * out[o] + 0.5 * (uc + dt * L[q][v]);
    }
  }
}

// --------------------------------------------------------- flux correction --
// One thread per (listed face of direction d, face cell): the list holds
// 2 slot + side of the coarse leaf faces whose neighbour region holds finer
// leaves; the coarse face's A F is replaced by the sum of the fine faces'
// A F.  coef: 1 after stage 1 (U1), 1/2 after stage 2 (U).  An edge or
// corner cell of a block lies on faces of several directions: one launch
// per direction keeps each cell's updates ordered (blocks have >= 4 cells a
// side, so the two faces of one direction never share a cell).
__global__ void __launch_bounds__(256) k_amr_reflux(AmrArgs a, const int* __restrict__ list,
                                                    int n, int stage, int d) {
  const int area = face_cells(a, d);
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (long long)area * n || !a.clock->active) return;
  const int ent = list[q / area];
  const int slot = ent >> 1, side = ent & 1;
  const int fq = (int)(q % area);
  const int* key = a.key + 4 * slot;
  const int l = key[0];
  if (l >= a.nlev) return;
  const int w2 = d == 0 ? a.bt : a.br;
  const int y = fq / w2, x = fq - y * w2;
  // the neighbour block of the same level across this face
  int nb[3] = {key[1], key[2], key[3]};
  nb[d] += side ? 1 : -1;
  const AmrLevel& L = a.lv[l];
  if (d == 2) nb[2] = (nb[2] + L.nbp) % L.nbp;
  if (d == 0 && (nb[0] < 0 || nb[0] >= L.nbr)) return;
  if (d == 1 && (nb[1] < 0 || nb[1] >= L.nbt)) return;
  const int ns = L.map[((long long)nb[2] * L.nbt + nb[1]) * L.nbr + nb[0]];
  if (ns < 0 || a.leaf[ns]) return;
  // coarse cell next to the face (block-local), its global indices
  int ci, cj, ck;
  if (d == 0) {
    ci = side ? a.br - 1 : 0;
    cj = x;
    ck = y;
  } else if (d == 1) {
    ci = x;
    cj = side ? a.bt - 1 : 0;
    ck = y;
  } else {
    ci = x;
    cj = y;
    ck = side ? a.bp - 1 : 0;
  }
  const int gi = key[1] * a.br + ci, gj = key[2] * a.bt + cj;
  const Metric<double>& m = L.m;
  const Metric<double>& mf = a.lv[l + 1].m;
  // coarse face area, and the fine faces (2 x 2) of the finer leaves
  double Ac;
  if (d == 0)
    Ac = (side ? m.rp2[gi] : m.rm2[gi]) / m.ict[gj] * L.dph;
  else if (d == 1)
    Ac = (side ? m.sp[gj] : m.sm[gj]) * m.hr[gi] / m.ivr[gi] * L.dph;
  else
    Ac = m.hr[gi] / m.ivr[gi] * L.dth;
  const double V = vol_nophi(a, l, gi, gj) * L.dph;
  const int face = 2 * d + side, fface = 2 * d + (1 - side);
  const double dt = a.clock->dt * (stage == 1 ? 1.0 : 0.5);
  double* tgt = stage == 1 ? a.U1 : a.U;
  const int gk = key[3] * a.bp + ck;
  // the 2 x 2 fine faces: slot, face cell and area (s = 2 s2 + s1)
  const AmrLevel& LF = a.lv[l + 1];
  int fsl[4], fqf[4];
  double Af[4];
  bool ok = true;
  for (int s = 0; s < 4; ++s) {
    const int s2 = s >> 1, s1 = s & 1;
    // fine cell indices (global, level l+1) on the fine side of the face
    int fi = 2 * gi, fj = 2 * gj, fk = 2 * gk;
    if (d == 0) {
      fi = side ? 2 * gi + 2 : 2 * gi - 1;
      fj += s1;
      fk += s2;
    } else if (d == 1) {
      fj = side ? 2 * gj + 2 : 2 * gj - 1;
      fi += s1;
      fk += s2;
    } else {
      fk = side ? 2 * gk + 2 : 2 * gk - 1;
      fi += s1;
      fj += s2;
    }
    if (d == 2) fk = (fk + LF.np) % LF.np;
    const int fs = amr_slot(a, l + 1, fi, fj, fk);
    fsl[s] = fs;
    fqf[s] = 0;
    Af[s] = 0.0;
    if (fs < 0) {  // cannot happen in a valid tree: poison the cell
      ok = false;
      continue;
    }
    const int* fkey = a.key + 4 * fs;
    const int li = fi - fkey[1] * a.br, lj = fj - fkey[2] * a.bt, lk = fk - fkey[3] * a.bp;
    if (d == 0) {
      fqf[s] = lk * a.bt + lj;
      Af[s] = (side ? mf.rm2[fi] : mf.rp2[fi]) / mf.ict[fj] * LF.dph;
    } else if (d == 1) {
      fqf[s] = lk * a.br + li;
      Af[s] = (side ? mf.sm[fj] : mf.sp[fj]) * mf.hr[fi] / mf.ivr[fi] * LF.dph;
    } else {
      fqf[s] = lj * a.br + li;
      Af[s] = mf.hr[fi] / mf.ivr[fi] * LF.dth;
    }
  }
  for (int v = 0; v < NA; ++v) {
    double sumf = 0.0;
    for (int s = 0; s < 4; ++s)
      if (fsl[s] >= 0) sumf += Af[s] * a.F[fidx(a, fsl[s], fface, v, fqf[s])];
    if (!ok) sumf = __builtin_nan("");
    const double delta = sumf - Ac * a.F[fidx(a, slot, face, v, fq)];
    const double dL = (side ? -delta : delta) / V;
    tgt[pidx(a, slot, v, AG + ck, AG + cj, AG + ci)] += dt * dL;
  }
}

// ------------------------------------------------------------------- CFL --
__global__ void __launch_bounds__(256) k_amr_cfl(AmrArgs a, const int* __restrict__ list) {
  const int slot = list[blockIdx.x];
  const int* key = a.key + 4 * slot;
  const int l = key[0];
  const Metric<double>& m = a.lv[l].m;
  double lam = 0.0;
  int bad = BAD_NONE;
  const int ncell = a.br * a.bt * a.bp;
  for (int c = threadIdx.x; c < ncell; c += blockDim.x) {
    const int ci = c % a.br, cj = (c / a.br) % a.bt, ck = c / (a.br * a.bt);
    double u[NV], w[NV];
    for (int v = 0; v < NV; ++v) u[v] = a.U[pidx(a, slot, v, AG + ck, AG + cj, AG + ci)];
    cons2prim<double>(u, w, a.gm1);
    const int gi = key[1] * a.br + ci, gj = key[2] * a.bt + cj;
    const double rate = cell_rate<double>(w, m, gi, gj, a.gam);
    lam = fmax(lam, rate);
    if (bad == BAD_NONE && !cell_valid<double>(u, w)) bad = slot * ncell + c;
  }
  write_partials(a.partials, blockIdx.x, lam, 0.0, 1.0, bad);
}

// ------------------------------------------------------------ indicators --
// Per listed leaf: max tau and max of -div(V) r / (2 |v_r|) (ghosts filled).
__global__ void __launch_bounds__(256) k_amr_indicators(AmrArgs a, const int* __restrict__ list,
                                                        double* __restrict__ out) {
  __shared__ double sh[2][4];
  const int slot = list[blockIdx.x];
  const int* key = a.key + 4 * slot;
  const int l = key[0];
  const Metric<double>& m = a.lv[l].m;
  double tmax = -1e300, cmax = -1e300;
  const int ncell = a.br * a.bt * a.bp;
  for (int c = threadIdx.x; c < ncell; c += blockDim.x) {
    const int ci = c % a.br, cj = (c / a.br) % a.bt, ck = c / (a.br * a.bt);
    const int ii = AG + ci, jj = AG + cj, kk = AG + ck;
    const int gi = key[1] * a.br + ci, gj = key[2] * a.bt + cj;
    auto vel = [&](int k2, int j2, int i2, int comp) {
      return a.U[pidx(a, slot, comp, k2, j2, i2)] / a.U[pidx(a, slot, 0, k2, j2, i2)];
    };
    const double v0r = vel(kk, jj, ii, 1), v0t = vel(kk, jj, ii, 2), v0p = vel(kk, jj, ii, 3);
    const double vr0 = 0.5 * (vel(kk, jj, ii - 1, 1) + v0r), vr1 = 0.5 * (v0r + vel(kk, jj, ii + 1, 1));
    const double vt0 = 0.5 * (vel(kk, jj - 1, ii, 2) + v0t), vt1 = 0.5 * (v0t + vel(kk, jj + 1, ii, 2));
    const double vp0 = 0.5 * (vel(kk - 1, jj, ii, 3) + v0p), vp1 = 0.5 * (v0p + vel(kk + 1, jj, ii, 3));
    const double div = (m.rp2[gi] * vr1 - m.rm2[gi] * vr0) * m.ivr[gi] +
                       m.hr[gi] * (m.sp[gj] * vt1 - m.sm[gj] * vt0) * m.ict[gj] +
                       m.hr[gi] * m.phf[gj] * (vp1 - vp0);
    const double comp = -div * m.rc[gi] / (2.0 * fabs(v0r));
    const double tau = a.U[pidx(a, slot, 8, kk, jj, ii)] / a.U[pidx(a, slot, 0, kk, jj, ii)];
    tmax = fmax(tmax, tau);
    cmax = fmax(cmax, comp);
  }
  for (int off = 32; off > 0; off >>= 1) {
    tmax = fmax(tmax, __shfl_xor(tmax, off, 64));
    cmax = fmax(cmax, __shfl_xor(cmax, off, 64));
  }
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[0][wv] = tmax;
    sh[1][wv] = cmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < (int)(blockDim.x >> 6); ++q) {
      tmax = fmax(tmax, sh[0][q]);
      cmax = fmax(cmax, sh[1][q]);
    }
    out[2 * blockIdx.x] = tmax;
    out[2 * blockIdx.x + 1] = cmax;
  }
}

// ------------------------------------------------- split, merge, init, io --
// pairs[2q] = parent slot, pairs[2q+1] = child slot: the child's cells from
// the parent's padded U (ghosts filled).
__global__ void __launch_bounds__(256) k_amr_prolong(AmrArgs a, const int* __restrict__ pairs) {
  const int ps = pairs[2 * blockIdx.x], cs = pairs[2 * blockIdx.x + 1];
  const int* pk = a.key + 4 * ps;
  const int* ck = a.key + 4 * cs;
  const int l = pk[0];
  const int ncell = a.br * a.bt * a.bp;
  for (int c = threadIdx.x; c < ncell; c += blockDim.x) {
    const int ci = c % a.br, cj = (c / a.br) % a.bt, cq = c / (a.br * a.bt);
    // global child cell and its coarse parent cell
    const int fi = ck[1] * a.br + ci, fj = ck[2] * a.bt + cj, fk = ck[3] * a.bp + cq;
    const int gi = fi >> 1, gj = fj >> 1, gk = fk >> 1;
    const int ii = AG + gi - pk[1] * a.br, jj = AG + gj - pk[2] * a.bt, kk = AG + gk - pk[3] * a.bp;
    const int sub = ((fk - 2 * gk) << 2) | ((fj - 2 * gj) << 1) | (fi - 2 * gi);
    for (int v = 0; v < NA; ++v) {
      const double c0 = a.U[pidx(a, ps, v, kk, jj, ii)];
      const double n[6] = {a.U[pidx(a, ps, v, kk, jj, ii - 1)], a.U[pidx(a, ps, v, kk, jj, ii + 1)],
                           a.U[pidx(a, ps, v, kk, jj - 1, ii)], a.U[pidx(a, ps, v, kk, jj + 1, ii)],
                           a.U[pidx(a, ps, v, kk - 1, jj, ii)], a.U[pidx(a, ps, v, kk + 1, jj, ii)]};
      double ch[8];
      prolong8(a, l, gi, gj, c0, n, ch);
      a.U[pidx(a, cs, v, AG + cq, AG + cj, AG + ci)] = ch[sub];
    }
  }
}

// parents[q]: the parent's cells from its 8 children (volume-weighted).
__global__ void __launch_bounds__(256) k_amr_restrict(AmrArgs a, const int* __restrict__ parents) {
  const int ps = parents[blockIdx.x];
  const int* pk = a.key + 4 * ps;
  const int l = pk[0];
  const int ncell = a.br * a.bt * a.bp;
  for (int c = threadIdx.x; c < ncell; c += blockDim.x) {
    const int ci = c % a.br, cj = (c / a.br) % a.bt, cq = c / (a.br * a.bt);
    const int gi = pk[1] * a.br + ci, gj = pk[2] * a.bt + cj, gk = pk[3] * a.bp + cq;
    double acc[NA], vs = 0.0;
    for (int v = 0; v < NA; ++v) acc[v] = 0.0;
    for (int s = 0; s < 8; ++s) {
      const int e = s >> 2, b = (s >> 1) & 1, cc = s & 1;
      const int fi = 2 * gi + cc, fj = 2 * gj + b, fk = 2 * gk + e;
      const int fs = l < a.nlev ? amr_slot(a, l + 1, fi, fj, fk) : -1;
      if (fs < 0) {  // cannot happen for a merge of 8 leaves
        vs = __builtin_nan("");
        continue;
      }
      const int* key = a.key + 4 * fs;
      const double vol = vol_nophi(a, l + 1, fi, fj);
      vs += vol;
      for (int v = 0; v < NA; ++v)
        acc[v] += a.U[pidx(a, fs, v, AG + fk - key[3] * a.bp, AG + fj - key[2] * a.bt,
                           AG + fi - key[1] * a.br)] * vol;
    }
    for (int v = 0; v < NA; ++v) a.U[pidx(a, ps, v, AG + cq, AG + cj, AG + ci)] = acc[v] / vs;
  }
}

// Level-1 leaves from the radial expansion of the first map (Sect. 2.1).
__global__ void __launch_bounds__(256) k_amr_init(AmrArgs a, const int* __restrict__ list,
                                                  double gam) {
  const int slot = list[blockIdx.x];
  const int* key = a.key + 4 * slot;
  const AmrLevel& L = a.lv[1];
  const long long plane = (long long)a.bnd.nt * a.bnd.np;
  const int ncell = a.br * a.bt * a.bp;
  for (int c = threadIdx.x; c < ncell; c += blockDim.x) {
    const int ci = c % a.br, cj = (c / a.br) % a.bt, cq = c / (a.br * a.bt);
    const int i = key[1] * a.br + ci, j = key[2] * a.bt + cj, k = key[3] * a.bp + cq;
    const double rc = L.m.rc[i];
    const double x = a.r_in / rc;
    const double sth = sin(L.m64[OFF_TC64(L.nr, L.nt) + j]);
    const long long q = (long long)j * a.bnd.np + k;
    double w[NV];
    w[0] = a.bnd.maps[0 * plane + q] * x * x;
    w[1] = a.bnd.maps[1 * plane + q];
    w[2] = 0.0;
    w[3] = -a.omega * rc * sth;
    w[4] = a.bnd.maps[4 * plane + q] * pow(x, 2.0 * gam);
    w[5] = a.bnd.maps[5 * plane + q] * x * x;
    w[6] = 0.0;
    w[7] = a.bnd.maps[7 * plane + q] * x;
    double u[NA];
    prim_to_cons9(a, w, 0.0, u);
    for (int v = 0; v < NA; ++v) a.U[pidx(a, slot, v, AG + cq, AG + cj, AG + ci)] = u[v];
  }
}

__global__ void k_amr_copy_out(AmrArgs a, int slot, double* __restrict__ out) {
  const int ncell = a.br * a.bt * a.bp;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < NA * ncell; c += gridDim.x * blockDim.x) {
    const int v = c / ncell, q = c - v * ncell;
    const int ci = q % a.br, cj = (q / a.br) % a.bt, cq = q / (a.br * a.bt);
    out[c] = a.U[pidx(a, slot, v, AG + cq, AG + cj, AG + ci)];
  }
}

}  // namespace icr

// ======================================================================
// Host side: the block tree, the step loop and the C-ABI.
// ======================================================================
using namespace icr;

namespace {

constexpr double kAUm = 1.495978707e11;
constexpr double kVu = 1.0e5;
constexpr double kMp = 1.67262192369e-27;
constexpr double kKb = 1.380649e-23;
constexpr double kMu0 = 4.0e-7 * 3.14159265358979323846;
constexpr double kGMs = 1.32712440018e20;
constexpr double kPI = 3.14159265358979323846;

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

struct Key {
  int l, i, j, k;
  bool operator<(const Key& o) const {
    if (l != o.l) return l < o.l;
    if (i != o.i) return i < o.i;
    if (j != o.j) return j < o.j;
    return k < o.k;
  }
  bool operator==(const Key& o) const { return l == o.l && i == o.i && j == o.j && k == o.k; }
};

int err(int code, const std::string& m) { return set_error(code, m.c_str()); }

#define AMR_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return err(ICR_ERR_HIP, std::string(#expr) + " failed: " +    \
                                                      hipGetErrorString(e_));           \
  } while (0)

struct AmrLayout {
  size_t U, U1, F, leaf, key, maps[AMR_MAXL + 1], m64[AMR_MAXL + 1], mr[AMR_MAXL + 1],
      bmaps, tau, cme, clock, partials, ind, lists, rlist, stage, total;
};

}  // namespace

struct icr_amr {
  icr_grid g;
  icr_phys p;
  icr_amr_params q;
  hipStream_t stream;
  char* ws;
  AmrLayout L;
  int nlev, pr, pt, pp, fmax;
  long long bvol;
  int nb[AMR_MAXL + 1][3];
  double t_unit, len_unit, rho_unit, p_unit, b_unit, v_unit, omega, r_in, gm;
  // tree
  std::map<Key, int> slot_of;      // every block (leaf or not) -> slot
  std::vector<Key> key_of;         // slot -> key
  std::vector<unsigned char> leaf; // slot -> leaf flag
  std::vector<int> hmap[AMR_MAXL + 1];  // level -> [nbp][nbt][nbr] slot or -1 (device copy: maps)
  std::vector<int> free_slots;
  int n_maps = 0, n_cme = 0;
  std::vector<double> tau_h;
  bool have_maps = false, have_state = false;
  long long steps_done = 0;

  char* at(size_t off) { return ws + off; }
  DevClock* clock() { return (DevClock*)at(L.clock); }

  AmrArgs args() {
    AmrArgs a;
    std::memset(&a, 0, sizeof a);
    a.U = (double*)at(L.U);
    a.U1 = (double*)at(L.U1);
    a.F = (double*)at(L.F);
    a.leaf = (const unsigned char*)at(L.leaf);
    a.key = (const int*)at(L.key);
    for (int l = 1; l <= nlev; ++l) {
      AmrLevel& v = a.lv[l];
      v.nr = nb[l][0] * q.block_r;
      v.nt = nb[l][1] * q.block_theta;
      v.np = nb[l][2] * q.block_phi;
      v.nbr = nb[l][0];
      v.nbt = nb[l][1];
      v.nbp = nb[l][2];
      v.dth = (g.th_max - g.th_min) / v.nt;
      v.dph = 2.0 * kPI / v.np;
      v.m = metric_view<double>((const double*)at(L.mr[l]), v.nr, v.nt, v.dth);
      v.m64 = (const double*)at(L.m64[l]);
      v.map = (const int*)at(L.maps[l]);
    }
    a.nlev = nlev;
    a.br = q.block_r;
    a.bt = q.block_theta;
    a.bp = q.block_phi;
    a.pr = pr;
    a.pt = pt;
    a.pp = pp;
    a.fmax = fmax;
    a.bvol = bvol;
    a.bnd.nt = g.n_theta;
    a.bnd.np = g.n_phi;
    a.bnd.n_maps = n_maps;
    a.bnd.tau = (const double*)at(L.tau);
    a.bnd.maps = (const double*)at(L.bmaps);
    a.bnd.n_cme = n_cme;
    a.bnd.cme = (const double*)at(L.cme);
    a.bnd.tc = (const double*)at(L.m64[1]) + OFF_TC64(g.n_r, g.n_theta);
    a.bnd.dph = 2.0 * kPI / g.n_phi;
    a.bnd.omega = omega;
    a.bnd.r_in = r_in;
    a.clock = clock();
    a.partials = (double*)at(L.partials);
    a.gam = p.gamma;
    a.gm1 = p.gamma - 1.0;
    a.igm1 = 1.0 / (p.gamma - 1.0);
    a.omega = omega;
    a.cfl = p.cfl;
    a.r_in = r_in;
    a.gravity = p.gravity ? 1 : 0;
    a.corot = p.corotation ? 1 : 0;
    return a;
  }

  std::vector<Key> leaves(int l = 0) const {
    std::vector<Key> out;
    for (const auto& kv : slot_of)
      if (leaf[kv.second] && (l == 0 || kv.first.l == l)) out.push_back(kv.first);
    return out;  // std::map order: level, i, j, k
  }
  size_t map_index(const Key& k) const {
    return ((size_t)k.k * nb[k.l][1] + k.j) * nb[k.l][0] + k.i;
  }
  // slot of a block, -1 where there is none (also outside the levels / grid)
  int slot(const Key& k) const {
    if (k.l < 1 || k.l > nlev || k.i < 0 || k.j < 0 || k.k < 0 || k.i >= nb[k.l][0] ||
        k.j >= nb[k.l][1] || k.k >= nb[k.l][2])
      return -1;
    return hmap[k.l][map_index(k)];
  }
  bool has(const Key& k) const { return slot(k) >= 0; }
  bool is_leaf(const Key& k) const {
    const int s = slot(k);
    return s >= 0 && leaf[s];
  }
  bool neighbour(const Key& k, int d, int side, Key* out) const {
    int b[3] = {k.i, k.j, k.k};
    b[d] += side ? 1 : -1;
    if (d == 2) {
      b[2] = (b[2] % nb[k.l][2] + nb[k.l][2]) % nb[k.l][2];
    } else if (b[d] < 0 || b[d] >= nb[k.l][d]) {
      return false;
    }
    *out = Key{k.l, b[0], b[1], b[2]};
    return true;
  }
  static Key parent(const Key& k) { return Key{k.l - 1, k.i / 2, k.j / 2, k.k / 2}; }
  static std::vector<Key> children(const Key& k) {
    std::vector<Key> c;
    for (int e = 0; e < 2; ++e)
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) c.push_back(Key{k.l + 1, 2 * k.i + a, 2 * k.j + b, 2 * k.k + e});
    return c;
  }

  int add_block(const Key& k) {
    if (free_slots.empty()) return -1;
    const int s = free_slots.back();
    free_slots.pop_back();
    slot_of[k] = s;
    hmap[k.l][map_index(k)] = s;
    key_of[s] = k;
    leaf[s] = 1;
    return s;
  }
  void remove_block(const Key& k) {
    const int s = slot_of.at(k);
    slot_of.erase(k);
    hmap[k.l][map_index(k)] = -1;
    leaf[s] = 0;
    free_slots.push_back(s);
  }

  // upload key table, leaf flags and level maps
  int upload_tree() {
    const int mb = q.max_blocks;
    std::vector<int> keys(4 * (size_t)mb, 0);
    for (const auto& kv : slot_of) {
      int* p4 = &keys[4 * (size_t)kv.second];
      p4[0] = kv.first.l;
      p4[1] = kv.first.i;
      p4[2] = kv.first.j;
      p4[3] = kv.first.k;
    }
    AMR_TRY(hipMemcpyAsync(at(L.key), keys.data(), keys.size() * sizeof(int),
                           hipMemcpyHostToDevice, stream));
    AMR_TRY(hipMemcpyAsync(at(L.leaf), leaf.data(), leaf.size(), hipMemcpyHostToDevice, stream));
    for (int l = 1; l <= nlev; ++l)
      AMR_TRY(hipMemcpyAsync(at(L.maps[l]), hmap[l].data(), hmap[l].size() * sizeof(int),
                             hipMemcpyHostToDevice, stream));
    AMR_TRY(hipStreamSynchronize(stream));
    return ICR_OK;
  }

  // device lists of slots: the leaves (all, and per level) are rebuilt after
  // every change of the tree; temporary lists go after them
  int n_all = 0, lvl_off[AMR_MAXL + 1] = {}, lvl_n[AMR_MAXL + 1] = {};
  int* list_at(size_t at_int) { return (int*)at(L.lists) + at_int; }
  int* upload_temp(const std::vector<int>& v) {
    int* d = list_at(2 * (size_t)q.max_blocks);
    if (!v.empty())
      (void)hipMemcpy(d, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice);
    return d;
  }
  int rebuild_lists() {
    std::vector<int> all = slots(leaves());
    n_all = (int)all.size();
    std::vector<int> per;
    for (int l = 1; l <= nlev; ++l) {
      std::vector<int> s = slots(leaves(l));
      lvl_off[l] = (int)per.size();
      lvl_n[l] = (int)s.size();
      per.insert(per.end(), s.begin(), s.end());
    }
    if (!all.empty())
      AMR_TRY(hipMemcpy(list_at(0), all.data(), all.size() * sizeof(int), hipMemcpyHostToDevice));
    if (!per.empty())
      AMR_TRY(hipMemcpy(list_at(q.max_blocks), per.data(), per.size() * sizeof(int),
                        hipMemcpyHostToDevice));
    // faces of leaves below the top level whose same-level neighbour is
    // refined (its children there are leaves, by the one-level rule)
    for (int d = 0; d < 3; ++d) {
      std::vector<int> e;
      for (const int sl : all) {
        const Key& k = key_of[sl];
        if (k.l >= nlev) continue;
        for (int side = 0; side < 2; ++side) {
          Key nk;
          if (!neighbour(k, d, side, &nk)) continue;
          const int ns = slot(nk);
          if (ns >= 0 && !leaf[ns]) e.push_back(2 * sl + side);
        }
      }
      n_rl[d] = (int)e.size();
      if (!e.empty())
        AMR_TRY(hipMemcpy(rlist_at(d), e.data(), e.size() * sizeof(int), hipMemcpyHostToDevice));
    }
    return ICR_OK;
  }
  int n_rl[3] = {0, 0, 0};
  int* rlist_at(int d) { return (int*)at(L.rlist) + (size_t)d * 2 * q.max_blocks; }

  std::vector<int> slots(const std::vector<Key>& ks) const {
    std::vector<int> s;
    for (const Key& k : ks) s.push_back(slot(k));
    return s;
  }

  template <int FLUX, int LIM>
  void launch_stage_t(const AmrArgs& a, int* d, int n, int stage) {
    const int br = q.block_r, bt = q.block_theta, bp = q.block_phi;
    const int nf = std::max((br + 1) * bt * bp, std::max(br * (bt + 1) * bp, br * bt * (bp + 1)));
    const size_t lds = sizeof(double) * NA * (size_t)nf;
    if (br * bt * bp <= AMR_FO_CELLS && lds <= 48 * 1024)
      hipLaunchKernelGGL((k_amr_stage_fo<FLUX, LIM>), dim3(n), dim3(256), lds, stream, a, d,
                         stage);
    else
      hipLaunchKernelGGL((k_amr_stage<FLUX, LIM>), dim3(n), dim3(256), 0, stream, a, d, stage);
  }
  void launch_stage(const AmrArgs& a, int* d, int n, int stage) {
    const int f = p.flux, lm = p.limiter;
    if (f == ICR_FLUX_TVDLF && lm == ICR_LIM_MINMOD) launch_stage_t<FLUX_TVDLF, LIM_MINMOD>(a, d, n, stage);
    else if (f == ICR_FLUX_TVDLF) launch_stage_t<FLUX_TVDLF, LIM_MC>(a, d, n, stage);
    else if (f == ICR_FLUX_HLL && lm == ICR_LIM_MINMOD) launch_stage_t<FLUX_HLL, LIM_MINMOD>(a, d, n, stage);
    else if (f == ICR_FLUX_HLL) launch_stage_t<FLUX_HLL, LIM_MC>(a, d, n, stage);
    else if (lm == ICR_LIM_MINMOD) launch_stage_t<FLUX_HLLD, LIM_MINMOD>(a, d, n, stage);
    else launch_stage_t<FLUX_HLLD, LIM_MC>(a, d, n, stage);
  }

  // stage right-hand sides, updates and flux corrections; CFL of the result
  void enqueue_step() {
    const size_t nl = (size_t)n_all;
    int* d_all = list_at(0);
    const long long area[3] = {(long long)q.block_phi * q.block_theta,
                               (long long)q.block_phi * q.block_r,
                               (long long)q.block_theta * q.block_r};
    for (int stage = 1; stage <= 2; ++stage) {
      fill_ghosts_at(stage == 2, stage == 2, 0);
      AmrArgs a = args();
      launch_stage(a, d_all, (int)nl, stage);
      for (int d = 0; d < 3; ++d) {
        if (n_rl[d] == 0) continue;
        const long long n = area[d] * (long long)n_rl[d];
        hipLaunchKernelGGL(k_amr_reflux, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                           a, rlist_at(d), n_rl[d], stage, d);
      }
    }
    AmrArgs a = args();
    hipLaunchKernelGGL(k_amr_cfl, dim3((unsigned)nl), dim3(256), 0, stream, a, d_all);
    ProbeArgs pa;
    std::memset(&pa, 0, sizeof pa);
    launch_finalize<double>(clock(), (const double*)at(L.partials), (int)nl, p.cfl, 1, 0, pa,
                            nullptr, nullptr, stream);
  }

  void fill_ghosts_at(int use_u1, int plus_dt, int always) {
    AmrArgs a = args();
    for (int l = 1; l <= nlev; ++l) {
      if (lvl_n[l] == 0) continue;
      int* d = list_at((size_t)q.max_blocks + lvl_off[l]);
      const long long per = 4LL * (q.block_phi * q.block_theta + q.block_phi * q.block_r +
                                   q.block_theta * q.block_r);
      const long long n = per * (long long)lvl_n[l];
      hipLaunchKernelGGL(k_amr_ghost, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, a,
                         l, d, lvl_n[l], use_u1, plus_dt, always);
    }
  }

  int first_dt() {
    int* d_all = list_at(0);
    AmrArgs a = args();
    hipLaunchKernelGGL(k_amr_cfl, dim3((unsigned)n_all), dim3(256), 0, stream, a, d_all);
    ProbeArgs pa;
    std::memset(&pa, 0, sizeof pa);
    launch_finalize<double>(clock(), (const double*)at(L.partials), n_all, p.cfl, 0, 0, pa,
                            nullptr, nullptr, stream);
    AMR_TRY(hipGetLastError());
    AMR_TRY(hipStreamSynchronize(stream));
    return ICR_OK;
  }

  int read_clock(DevClock* c) {
    AMR_TRY(hipMemcpyAsync(c, clock(), sizeof(DevClock), hipMemcpyDeviceToHost, stream));
    AMR_TRY(hipStreamSynchronize(stream));
    return ICR_OK;
  }
  int write_clock(const DevClock* c) {
    AMR_TRY(hipMemcpyAsync(clock(), c, sizeof(DevClock), hipMemcpyHostToDevice, stream));
    AMR_TRY(hipStreamSynchronize(stream));
    return ICR_OK;
  }

  // --- regrid ------------------------------------------------------------
  void balance(std::set<Key>& refine) const {
    bool changed = true;
    while (changed) {
      changed = false;
      std::vector<Key> cur(refine.begin(), refine.end());
      for (const Key& k : cur)
        for (int d = 0; d < 3; ++d)
          for (int s = 0; s < 2; ++s) {
            Key nk;
            if (!neighbour(k, d, s, &nk) || has(nk)) continue;
            const Key pk = parent(nk);
            if (is_leaf(pk) && !refine.count(pk)) {
              refine.insert(pk);
              changed = true;
            }
          }
    }
  }

  int apply(const std::set<Key>& coarsen, const std::set<Key>& refine) {
    // ghosts of U at the current time for the prolongation slopes
    fill_ghosts_at(0, 0, 1);
    // merges: parents take the volume-weighted mean of their children
    std::vector<int> parents;
    for (const Key& pk : coarsen) parents.push_back(slot_of.at(pk));
    if (!parents.empty()) {
      int* d = upload_temp(parents);
      AmrArgs a = args();
      hipLaunchKernelGGL(k_amr_restrict, dim3((unsigned)parents.size()), dim3(256), 0, stream, a,
                         d);
      AMR_TRY(hipStreamSynchronize(stream));
      for (const Key& pk : coarsen) {
        for (const Key& c : children(pk)) remove_block(c);
        leaf[slot_of.at(pk)] = 1;
      }
    }
    // splits, coarser levels first (std::set order is level-major)
    std::vector<int> pairs;
    for (const Key& k : refine) {
      if (!is_leaf(k)) continue;
      for (const Key& c : children(k)) {
        const int s = add_block(c);
        if (s < 0) return err(ICR_ERR_STATE, "AMR block pool full (raise max_blocks)");
        pairs.push_back(slot_of.at(k));
        pairs.push_back(s);
      }
      leaf[slot_of.at(k)] = 0;
    }
    int rc = upload_tree();
    if (!rc) rc = rebuild_lists();
    if (rc) return rc;
    if (!pairs.empty()) {
      // a split's children read their parent's padded block, which is not
      // touched by any other split of this pass (parents are distinct)
      int* d = upload_temp(pairs);
      AmrArgs a = args();
      hipLaunchKernelGGL(k_amr_prolong, dim3((unsigned)(pairs.size() / 2)), dim3(256), 0, stream,
                         a, d);
      AMR_TRY(hipGetLastError());
      AMR_TRY(hipStreamSynchronize(stream));
    }
    return ICR_OK;
  }

  int regrid() {
    std::vector<Key> lv = leaves();  // the order of the device list
    fill_ghosts_at(0, 0, 1);
    AmrArgs a = args();
    double* ind = (double*)at(L.ind);
    hipLaunchKernelGGL(k_amr_indicators, dim3((unsigned)n_all), dim3(256), 0, stream, a,
                       list_at(0), ind);
    std::vector<double> h(2 * lv.size());
    AMR_TRY(hipMemcpyAsync(h.data(), ind, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                           stream));
    AMR_TRY(hipStreamSynchronize(stream));
    // per slot: -1 not a leaf of this regrid, else the leaf's criterion
    std::vector<signed char> flag(q.max_blocks, -1);
    std::set<Key> refine;
    for (size_t n = 0; n < lv.size(); ++n) {
      const bool tr = h[2 * n] >= q.tau_threshold;
      const bool sh = h[2 * n + 1] >= q.shock_threshold;
      const bool f = q.criterion == ICR_AMR_TRACING ? tr : (q.criterion == ICR_AMR_SHOCK ? sh : (tr || sh));
      flag[slot(lv[n])] = f ? 1 : 0;
      if (f && lv[n].l < nlev) refine.insert(lv[n]);
    }
    balance(refine);
    std::set<Key> coarsen;
    std::set<Key> parents;
    for (const Key& k : lv)
      if (k.l > 1) parents.insert(parent(k));
    for (const Key& pk : parents) {
      bool all = true;
      for (const Key& c : children(pk)) {
        const int cs = slot(c);
        if (cs < 0 || !leaf[cs] || flag[cs] != 0 || refine.count(c)) all = false;
      }
      if (!all) continue;
      bool ok = true;
      for (int dd = 0; dd < 3; ++dd)
        for (int sd = 0; sd < 2; ++sd) {
          Key nk;
          if (!neighbour(pk, dd, sd, &nk)) continue;
          if (has(nk) && !is_leaf(nk))
            for (const Key& gch : children(nk))
              if (has(gch) && !is_leaf(gch)) ok = false;
          if (refine.count(nk)) ok = false;
          if (has(nk))
            for (const Key& gch : children(nk))
              if (refine.count(gch)) ok = false;
        }
      if (ok) coarsen.insert(pk);
    }
    return apply(coarsen, refine);
  }
};

namespace {

int validate_amr(const icr_grid* g, const icr_phys* p, const icr_amr_params* q) {
  if (!g || !p || !q) return err(ICR_ERR_ARG, "grid, phys and params must not be NULL");
  if (p->precision != ICR_PREC_F64) return err(ICR_ERR_UNSUPPORTED, "AMR runs in FP64 only");
  if (p->limiter == ICR_LIM_WENO5) return err(ICR_ERR_UNSUPPORTED, "AMR has two ghost layers (no WENO5)");
  if (p->bc_transverse != ICR_BCT_MAP) return err(ICR_ERR_UNSUPPORTED, "AMR uses the map transverse rule");
  if (q->block_r < 4 || q->block_theta < 4 || q->block_phi < 4)
    return err(ICR_ERR_ARG, "AMR blocks need at least 4 cells per side");
  if (g->n_r % q->block_r || g->n_theta % q->block_theta || g->n_phi % q->block_phi)
    return err(ICR_ERR_ARG, "the block size must divide the base grid");
  if (q->max_level < 1 || q->max_level > AMR_MAXL)
    return err(ICR_ERR_ARG, "max_level must be in [1, 6]");
  if (q->criterion < ICR_AMR_TRACING || q->criterion > ICR_AMR_COMBINED)
    return err(ICR_ERR_ARG, "unknown AMR criterion");
  if (q->regrid_every < 1) return err(ICR_ERR_ARG, "regrid_every must be >= 1");
  const long long base = (long long)(g->n_r / q->block_r) * (g->n_theta / q->block_theta) *
                         (g->n_phi / q->block_phi);
  if (q->max_blocks < base) return err(ICR_ERR_ARG, "max_blocks below the base grid's blocks");
  if (!(p->gamma > 1.0) || !(p->cfl > 0.0 && p->cfl <= 1.0)) return err(ICR_ERR_ARG, "gamma / cfl");
  if (!(g->r_in > 0 && g->r_out > g->r_in) || !(g->th_min > 0 && g->th_max > g->th_min && g->th_max < kPI))
    return err(ICR_ERR_ARG, "invalid grid extent");
  if (g->max_maps < 1 || g->max_cmes < 0) return err(ICR_ERR_ARG, "invalid capacities");
  return ICR_OK;
}

AmrLayout amr_layout(const icr_grid& g, const icr_amr_params& q) {
  AmrLayout L{};
  const long long pr = q.block_r + 2 * AG, pt = q.block_theta + 2 * AG, pp = q.block_phi + 2 * AG;
  const size_t bvol = (size_t)(pr * pt * pp);
  const int fmax = std::max(q.block_phi * q.block_theta,
                            std::max(q.block_phi * q.block_r, q.block_theta * q.block_r));
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off += al256(b);
    return o;
  };
  const size_t mb = (size_t)q.max_blocks;
  L.U = take(sizeof(double) * NA * bvol * mb);
  L.U1 = take(sizeof(double) * NA * bvol * mb);
  L.F = take(sizeof(double) * 6 * NA * (size_t)fmax * mb);
  L.leaf = take(mb);
  L.key = take(sizeof(int) * 4 * mb);
  for (int l = 1; l <= q.max_level; ++l) {
    const long long f = 1LL << (l - 1);
    const long long nr = g.n_r * f, nt = g.n_theta * f, np = g.n_phi * f;
    L.maps[l] = take(sizeof(int) * (size_t)((nr / q.block_r) * (nt / q.block_theta) *
                                            (np / q.block_phi)));
    L.m64[l] = take(sizeof(double) * (size_t)METRIC64_LEN((int)nr, (int)nt));
    L.mr[l] = take(sizeof(double) * (size_t)METRICR_LEN((int)nr, (int)nt));
  }
  L.bmaps = take(sizeof(double) * (size_t)g.max_maps * NV * g.n_theta * g.n_phi);
  L.tau = take(sizeof(double) * (size_t)g.max_maps);
  L.cme = take(sizeof(double) * 8 * (size_t)std::max(1, g.max_cmes));
  L.clock = take(sizeof(DevClock));
  L.partials = take(sizeof(double) * 4 * mb);
  L.ind = take(sizeof(double) * 2 * mb);
  // device lists: all leaves [mb], per-level leaves [mb], temporary [4 mb]
  L.lists = take(sizeof(int) * 6 * mb);
  // flux-correction lists: per direction, (slot, side) of the coarse leaf
  // faces next to finer leaves [2 mb] each
  L.rlist = take(sizeof(int) * 6 * mb);
  L.stage = take(sizeof(double) * NA * (size_t)q.block_r * q.block_theta * q.block_phi);
  L.total = off;
  return L;
}

}  // namespace

extern "C" {

int icr_amr_workspace_bytes(const icr_grid* g, const icr_phys* p, const icr_amr_params* q,
                            size_t* bytes) {
  int rc = validate_amr(g, p, q);
  if (rc) return rc;
  if (!bytes) return err(ICR_ERR_ARG, "bytes is NULL");
  *bytes = amr_layout(*g, *q).total;
  return ICR_OK;
}

int icr_amr_create(const icr_grid* g, const icr_phys* p, const icr_amr_params* q, void* ws,
                   size_t bytes, void* stream, icr_amr** out) {
  int rc = validate_amr(g, p, q);
  if (rc) return rc;
  if (!out) return err(ICR_ERR_ARG, "out is NULL");
  *out = nullptr;
  AmrLayout L = amr_layout(*g, *q);
  if (!ws || bytes < L.total) return err(ICR_ERR_ARG, "workspace too small");
  if (((uintptr_t)ws & 255) != 0) return err(ICR_ERR_ARG, "workspace must be 256-byte aligned");
  icr_amr* a = new icr_amr();
  a->g = *g;
  a->p = *p;
  a->q = *q;
  a->stream = (hipStream_t)stream;
  a->ws = (char*)ws;
  a->L = L;
  a->nlev = q->max_level;
  a->pr = q->block_r + 2 * AG;
  a->pt = q->block_theta + 2 * AG;
  a->pp = q->block_phi + 2 * AG;
  a->bvol = (long long)a->pr * a->pt * a->pp;
  a->fmax = std::max(q->block_phi * q->block_theta,
                     std::max(q->block_phi * q->block_r, q->block_theta * q->block_r));
  a->len_unit = kAUm;
  a->v_unit = kVu;
  a->t_unit = kAUm / kVu;
  a->rho_unit = kMp * 1.0e6;
  a->p_unit = a->rho_unit * kVu * kVu;
  a->b_unit = std::sqrt(kMu0 * a->rho_unit) * kVu;
  a->omega = p->corotation ? p->omega * a->t_unit : 0.0;
  a->r_in = g->r_in / a->len_unit;
  a->gm = p->gravity ? kGMs / (a->len_unit * kVu * kVu) : 0.0;
  for (int l = 1; l <= a->nlev; ++l) {
    const int f = 1 << (l - 1);
    a->nb[l][0] = g->n_r * f / q->block_r;
    a->nb[l][1] = g->n_theta * f / q->block_theta;
    a->nb[l][2] = g->n_phi * f / q->block_phi;
    MetricArgs m;
    m.nr = g->n_r * f;
    m.nt = g->n_theta * f;
    m.r_in = a->r_in;
    m.r_out = g->r_out / a->len_unit;
    m.q = std::pow(m.r_out / m.r_in, 1.0 / m.nr);
    m.th_min = g->th_min;
    m.th_max = g->th_max;
    m.dph = 2.0 * kPI / (g->n_phi * f);
    m.gm = a->gm;
    m.m64 = (double*)a->at(L.m64[l]);
    launch_metric(m, a->at(L.mr[l]), false, a->stream);
  }
  for (int l = 1; l <= a->nlev; ++l)
    a->hmap[l].assign((size_t)a->nb[l][0] * a->nb[l][1] * a->nb[l][2], -1);
  a->key_of.assign(q->max_blocks, Key{0, 0, 0, 0});
  a->leaf.assign(q->max_blocks, 0);
  for (int s = q->max_blocks - 1; s >= 0; --s) a->free_slots.push_back(s);
  for (int k = 0; k < a->nb[1][2]; ++k)
    for (int j = 0; j < a->nb[1][1]; ++j)
      for (int i = 0; i < a->nb[1][0]; ++i) a->add_block(Key{1, i, j, k});
  DevClock c;
  std::memset(&c, 0, sizeof c);
  c.bad = BAD_NONE;
  c.t_end = -1.0;
  c.last_sample = -1;
  rc = a->write_clock(&c);
  if (!rc) rc = a->upload_tree();
  if (!rc) rc = a->rebuild_lists();
  if (rc) {
    delete a;
    return rc;
  }
  *out = a;
  return ICR_OK;
}

void icr_amr_destroy(icr_amr* a) {
  if (!a) return;
  (void)hipStreamSynchronize(a->stream);
  delete a;
}

int icr_amr_set_boundary_maps(icr_amr* a, int n, const double* t_s, const double* maps) {
  if (!a || !t_s || !maps) return err(ICR_ERR_ARG, "NULL argument");
  if (n < 1 || n > a->g.max_maps) return err(ICR_ERR_ARG, "n_maps outside [1, max_maps]");
  for (int m = 1; m < n; ++m)
    if (!(t_s[m] > t_s[m - 1])) return err(ICR_ERR_ARG, "map times must ascend strictly");
  const size_t plane = (size_t)a->g.n_theta * a->g.n_phi;
  std::vector<double> h((size_t)n * NV * plane);
  const double sc[NV] = {a->rho_unit, a->v_unit, a->v_unit, a->v_unit,
                         a->p_unit,   a->b_unit, a->b_unit, a->b_unit};
  for (int m = 0; m < n; ++m)
    for (int v = 0; v < NV; ++v)
      for (size_t qq = 0; qq < plane; ++qq) {
        const double x = maps[((size_t)m * NV + v) * plane + qq];
        if ((v == 0 || v == 4) && !(x > 0.0)) return err(ICR_ERR_ARG, "map rho or p <= 0");
        if (!std::isfinite(x)) return err(ICR_ERR_ARG, "map has a non-finite value");
        h[((size_t)m * NV + v) * plane + qq] = x / sc[v];
      }
  std::vector<double> tau(n);
  for (int m = 0; m < n; ++m) tau[m] = t_s[m] / a->t_unit;
  AMR_TRY(hipMemcpyAsync(a->at(a->L.bmaps), h.data(), h.size() * sizeof(double),
                         hipMemcpyHostToDevice, a->stream));
  AMR_TRY(hipMemcpyAsync(a->at(a->L.tau), tau.data(), n * sizeof(double), hipMemcpyHostToDevice,
                         a->stream));
  AMR_TRY(hipStreamSynchronize(a->stream));
  a->n_maps = n;
  a->have_maps = true;
  return ICR_OK;
}

int icr_amr_set_cmes(icr_amr* a, int n, const double* rows) {
  if (!a) return err(ICR_ERR_ARG, "NULL argument");
  if (n < 0 || n > a->g.max_cmes) return err(ICR_ERR_ARG, "n outside [0, max_cmes]");
  if (n > 0 && !rows) return err(ICR_ERR_ARG, "rows is NULL");
  std::vector<double> c((size_t)8 * std::max(1, n));
  for (int k = 0; k < n; ++k) {
    const double* r = rows + 8 * k;
    if (!(r[1] > 0 && r[4] > 0 && r[5] > 0 && r[6] > 0 && r[7] > 0))
      return err(ICR_ERR_ARG, "CME duration, half-width, speed, density, T must be > 0");
    double* d = c.data() + 8 * k;
    d[0] = r[0] / a->t_unit;
    d[1] = r[1] / a->t_unit;
    d[2] = 0.5 * kPI - r[2];
    d[3] = r[3];
    d[4] = std::cos(r[4]);
    d[5] = r[5] / a->v_unit;
    d[6] = r[6] / a->rho_unit;
    d[7] = 2.0 * (r[6] / kMp) * kKb * r[7] / a->p_unit;
  }
  if (n > 0) {
    AMR_TRY(hipMemcpyAsync(a->at(a->L.cme), c.data(), 8 * n * sizeof(double),
                           hipMemcpyHostToDevice, a->stream));
    AMR_TRY(hipStreamSynchronize(a->stream));
  }
  a->n_cme = n;
  return ICR_OK;
}

int icr_amr_init_radial(icr_amr* a) {
  if (!a) return err(ICR_ERR_ARG, "NULL argument");
  if (!a->have_maps) return err(ICR_ERR_STATE, "set boundary maps first");
  // back to the base blocks
  std::vector<Key> all;
  for (const auto& kv : a->slot_of) all.push_back(kv.first);
  for (const Key& k : all)
    if (k.l > 1) a->remove_block(k);
  for (auto& kv : a->slot_of) a->leaf[kv.second] = 1;
  int rc = a->upload_tree();
  if (!rc) rc = a->rebuild_lists();
  if (rc) return rc;
  AmrArgs args = a->args();
  hipLaunchKernelGGL(k_amr_init, dim3((unsigned)a->n_all), dim3(256), 0, a->stream, args,
                     a->list_at(0), a->p.gamma);
  AMR_TRY(hipGetLastError());
  DevClock c;
  rc = a->read_clock(&c);
  if (rc) return rc;
  c.t = 0.0;
  c.step = 0;
  c.bad = BAD_NONE;
  c.last_dt = 0.0;
  c.resid = 0.0;
  rc = a->write_clock(&c);
  if (rc) return rc;
  a->have_state = true;
  a->steps_done = 0;
  return a->first_dt();
}

int icr_amr_step(icr_amr* a, int n, double t_end_s, icr_step_info* info) {
  if (!a) return err(ICR_ERR_ARG, "NULL argument");
  if (n < 0) return err(ICR_ERR_ARG, "n_steps must be >= 0");
  if (!a->have_state) return err(ICR_ERR_STATE, "initialise the state first");
  launch_clock_begin(a->clock(), t_end_s > 0.0 ? t_end_s / a->t_unit : -1.0, a->stream);
  DevClock c;
  for (int s = 0; s < n; ++s) {
    a->enqueue_step();
    ++a->steps_done;
    if (a->nlev > 1 && a->steps_done % a->q.regrid_every == 0) {
      int rc = a->read_clock(&c);
      if (rc) return rc;
      if (c.bad != BAD_NONE || !c.active) break;
      rc = a->regrid();
      if (rc) return rc;
      rc = a->first_dt();  // the CFL dt of the new leaves
      if (rc) return rc;
    }
  }
  AMR_TRY(hipGetLastError());
  int rc = a->read_clock(&c);
  if (rc) return rc;
  if (info) {
    info->steps_taken = (int)c.taken;
    info->status = c.bad == BAD_NONE ? ICR_OK : ICR_ERR_NONPHYSICAL;
    info->bad_cell = c.bad == BAD_NONE ? -1 : c.bad;
    info->t = c.t * a->t_unit;
    info->last_dt = c.last_dt * a->t_unit;
    info->residual = 0.0;
  }
  if (c.bad != BAD_NONE) return err(ICR_ERR_NONPHYSICAL, "non-physical cell on the refined grid");
  return ICR_OK;
}

int icr_amr_force_refine(icr_amr* a, int n, const int* keys) {
  if (!a || (n > 0 && !keys)) return err(ICR_ERR_ARG, "NULL argument");
  if (!a->have_state) return err(ICR_ERR_STATE, "initialise the state first");
  std::set<Key> refine;
  for (int q = 0; q < n; ++q) {
    const Key k{keys[4 * q], keys[4 * q + 1], keys[4 * q + 2], keys[4 * q + 3]};
    if (!a->is_leaf(k) || k.l >= a->nlev) return err(ICR_ERR_ARG, "not a leaf below the top level");
    refine.insert(k);
  }
  a->balance(refine);
  int rc = a->apply(std::set<Key>(), refine);
  if (rc) return rc;
  return a->first_dt();
}

int icr_amr_leaves(icr_amr* a, int cap, int* keys, int* n) {
  if (!a || !n) return err(ICR_ERR_ARG, "NULL argument");
  std::vector<Key> lv = a->leaves();
  *n = (int)lv.size();
  for (int q = 0; q < (int)lv.size() && q < cap; ++q) {
    keys[4 * q] = lv[q].l;
    keys[4 * q + 1] = lv[q].i;
    keys[4 * q + 2] = lv[q].j;
    keys[4 * q + 3] = lv[q].k;
  }
  return ICR_OK;
}

int icr_amr_get_block(icr_amr* a, const int* key, double* out) {
  if (!a || !key || !out) return err(ICR_ERR_ARG, "NULL argument");
  const Key k{key[0], key[1], key[2], key[3]};
  if (!a->is_leaf(k)) return err(ICR_ERR_ARG, "no such leaf");
  const int ncell = a->q.block_r * a->q.block_theta * a->q.block_phi;
  double* st = (double*)a->at(a->L.stage);
  AmrArgs args = a->args();
  hipLaunchKernelGGL(k_amr_copy_out, dim3(16), dim3(256), 0, a->stream, args, a->slot_of.at(k),
                     st);
  AMR_TRY(hipMemcpyAsync(out, st, sizeof(double) * NA * ncell, hipMemcpyDeviceToHost, a->stream));
  AMR_TRY(hipStreamSynchronize(a->stream));
  return ICR_OK;
}

int icr_amr_get_clock(icr_amr* a, icr_clock* out) {
  if (!a || !out) return err(ICR_ERR_ARG, "NULL argument");
  DevClock c;
  int rc = a->read_clock(&c);
  if (rc) return rc;
  out->t = c.t * a->t_unit;
  out->step = c.step;
  out->last_dt = c.last_dt * a->t_unit;
  out->next_dt = c.dt_cfl * a->t_unit;
  out->residual = 0.0;
  out->t_code = c.t;
  return ICR_OK;
}

}  // extern "C"
