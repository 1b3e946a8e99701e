/*
 * orc_mhd.c -- plain FP64 CPU oracle for the ideal-MHD heliosphere update.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the bench's CPU
 * baseline leg use it.  It shares no code with the HIP library.
 *
 * What it computes (Icarus 3.0, arXiv 2501.15923):
 *   - the ideal-MHD conservation laws for rho, rho*v, e, B in the frame
 *     co-rotating with the Sun: Sect. 2, Eqs. (1)-(4), total pressure Eq. (6),
 *     mu0 = 1 code units, gamma = 1.5, gravity and the centrifugal/Coriolis
 *     force F with its energy source v.F (Sect. 2, text after Eq. (6));
 *   - the 0.1 AU inner boundary taken from primitive-variable boundary maps
 *     (Sect. 2.1), the same value put in every ghost layer (Sect. 2.1, last
 *     paragraph), linear interpolation in time between successive maps
 *     (Sect. 3), and cone-CME overwrite of only the points inside the cone
 *     (Sect. 3.2, bc_icarus);
 *   - the initial state by radial expansion of the first map (Sect. 2.1);
 *   - edges the paper does not state: zero-gradient outflow at r_out,
 *     reflecting colatitude edges, periodic longitude;
 *   - sampling of the solution at moving locations interpolated from
 *     trajectory tables on the radially stretched grid (Sect. 2).
 * The paper does not print the finite-volume scheme; the reading used here
 * (primitive MUSCL with minmod/MC, TVDLF or HLL face fluxes, exact
 * finite-volume spherical divergence with area-difference pressure sources,
 * SSP-RK2, a max-sum CFL rule) is stated function by function below.
 *
 * Written for clarity, not speed: every array carries two ghost layers on
 * every side, every face flux is computed once per stage from face states
 * and stored, and nothing is fused.  Build with -O2 -ffp-contract=off.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NV 8 /* rho, m_r, m_t, m_p, e, B_r, B_t, B_p (or rho, v.., p, B..) */
/* ghost layers on each side: 2 for the slope-limited reconstructions, 3
 * for WENO5 (c->ng) */

/* ---- units: code = SI / unit --------------------------------------------- */
static const double AU_M = 1.495978707e11;      /* length unit [m]       */
static const double V_UNIT = 1.0e5;             /* velocity unit [m/s]   */
static const double M_PROTON = 1.67262192369e-27;
static const double K_BOLTZ = 1.380649e-23;
static const double MU0_SI = 4.0e-7 * 3.14159265358979323846;
static const double GM_SUN = 1.32712440018e20;  /* [m^3 s^-2] */

static double u_len(void) { return AU_M; }
static double u_time(void) { return AU_M / V_UNIT; }
static double u_rho(void) { return M_PROTON * 1.0e6; } /* 1 proton per cm^3 */
static double u_pres(void) { return u_rho() * V_UNIT * V_UNIT; }
static double u_bfield(void) { return sqrt(MU0_SI * u_rho()) * V_UNIT; }

enum { GEOM_SPH = 0, GEOM_SLAB = 1 };
enum { FLUX_TVDLF = 0, FLUX_HLL = 1, FLUX_HLLD = 2 };
enum { LIM_MINMOD = 0, LIM_MC = 1, LIM_WENO5 = 2 };
enum { BCT_MAP = 0, BCT_ASYMM = 1 };
enum { BCM_DRIVEN = 0, BCM_FROZEN = 1 };
enum { SLABX_OUTFLOW = 0, SLABX_PERIODIC = 1 };

typedef struct {
  int nr, nt, np;  /* active cells along r(x), theta(y), phi(z) */
  int ng;          /* ghost layers on each side */
  int gr, gt, gp;  /* padded sizes n + 2*ng */
  int geom, flux, limiter, gravity, corot, bc_transverse, bc_mode, slab_bcx;
  double gamma, omega, gm, cfl; /* code units */
  /* edges of the active cells (n+1 each), code units / radians */
  double *re, *te, *pe;
  /* cell centres of the active cells */
  double *rc, *tc, *pc;
  /* state with ghosts: U[v][k][j][i], i fastest */
  double *U;
  double t;     /* code time */
  long step;
  double last_dt, last_resid;
  double bflux[NV]; /* boundary-face integral of the last step, per variable */
  /* boundary maps (primitive, code units) */
  int n_maps;
  double *tau;  /* [n_maps] */
  double *maps; /* [n_maps][NV][nt][np] */
  /* cone CMEs: t0, dur, colat, lon, half-width, v, rho, p  (code units) */
  int n_cme;
  double *cme;
  /* per-axis metric factors (spherical), see build_metric() */
  double *volr, *hr, *garea, *ct, *se, *st, *snc, *csc;
  /* scratch */
  double *W, *F, *L, *U0, *U1;
  /* passive CME tracer (optional): conserved rho*tau with ghosts, its stage
   * copies and right-hand side, the upwind tau of every padded cell, and the
   * tracer's boundary-face integral of the last step */
  int tracer;
  double *T, *T0, *T1, *LT, *P, *FT;
  double tbflux;
} orc_ctx;

static size_t pad_cells(const orc_ctx *c) {
  return (size_t)c->gr * c->gt * c->gp;
}
/* index into a padded array; i, j, k are active-cell indices (may be <0). */
static size_t IX(const orc_ctx *c, int v, int i, int j, int k) {
  return (((size_t)v * c->gp + (k + c->ng)) * c->gt + (j + c->ng)) * c->gr + (i + c->ng);
}

/* ---- state conversions: Eq. (6) with mu0 = 1 ----------------------------- */
static void cons_to_prim(double gam, const double *u, double *w) {
  double rho = u[0];
  double vr = u[1] / rho, vt = u[2] / rho, vp = u[3] / rho;
  double kin = 0.5 * rho * (vr * vr + vt * vt + vp * vp);
  double mag = 0.5 * (u[5] * u[5] + u[6] * u[6] + u[7] * u[7]);
  w[0] = rho;
  w[1] = vr;
  w[2] = vt;
  w[3] = vp;
  w[4] = (gam - 1.0) * (u[4] - kin - mag);
  w[5] = u[5];
  w[6] = u[6];
  w[7] = u[7];
}

static void prim_to_cons(double gam, const double *w, double *u) {
  double rho = w[0];
  double kin = 0.5 * rho * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]);
  double mag = 0.5 * (w[5] * w[5] + w[6] * w[6] + w[7] * w[7]);
  u[0] = rho;
  u[1] = rho * w[1];
  u[2] = rho * w[2];
  u[3] = rho * w[3];
  u[4] = w[4] / (gam - 1.0) + kin + mag;
  u[5] = w[5];
  u[6] = w[6];
  u[7] = w[7];
}

/* Fast magnetosonic speed along the unit direction n (component index
 * 1..3 of the local orthonormal basis):
 *   c_f^2 = 1/2 [ a^2 + b^2 + sqrt((a^2+b^2)^2 - 4 a^2 B_n^2/rho) ],
 * a^2 = gamma p / rho, b^2 = |B|^2 / rho. */
static double fast_speed(double gam, const double *w, int n) {
  double rho = w[0];
  double a2 = gam * w[4] / rho;
  double b2 = (w[5] * w[5] + w[6] * w[6] + w[7] * w[7]) / rho;
  double bn = w[4 + n];
  double s = a2 + b2;
  double disc = s * s - 4.0 * a2 * bn * bn / rho;
  if (disc < 0.0) disc = 0.0;
  return sqrt(0.5 * (s + sqrt(disc)));
}

/* Physical flux of Eqs. (1)-(4) through a face with unit normal along local
 * component n: rho v_n; rho v_n v + p_tot e_n - B_n B; (e + p_tot) v_n -
 * B_n (v.B); v_n B - B_n v. */
static void phys_flux(double gam, const double *w, const double *u, int n,
                      double *f) {
  double vn = w[n], bn = w[4 + n];
  double b2 = w[5] * w[5] + w[6] * w[6] + w[7] * w[7];
  double ptot = w[4] + 0.5 * b2;
  double vb = w[1] * w[5] + w[2] * w[6] + w[3] * w[7];
  (void)gam;
  f[0] = w[0] * vn;
  for (int d = 1; d <= 3; ++d) {
    f[d] = u[d] * vn - bn * w[4 + d];
    if (d == n) f[d] += ptot;
  }
  f[4] = (u[4] + ptot) * vn - bn * vb;
  for (int d = 1; d <= 3; ++d) f[4 + d] = vn * w[4 + d] - bn * w[d];
}

/* WENO5 (Jiang & Shu 1996) value at the face between cells c and d from
 * the five cells a..e: the three third-order candidates of the stencils
 * ending at c, centred on c and starting at c, blended with weights
 * d_k / (eps + beta_k)^2 (d = 1/10, 6/10, 3/10) where beta_k measures each
 * candidate's smoothness.  eps is relative to the stencil's magnitude
 * (1e-6 of the mean square, plus 1e-40), so the weights do not depend on
 * the units of the variable. */
static double weno5(double a, double b, double c, double d, double e) {
  double q0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0;
  double q1 = (-b + 5.0 * c + 2.0 * d) / 6.0;
  double q2 = (2.0 * c + 5.0 * d - e) / 6.0;
  double b0 = 13.0 / 12.0 * (a - 2.0 * b + c) * (a - 2.0 * b + c) +
              0.25 * (a - 4.0 * b + 3.0 * c) * (a - 4.0 * b + 3.0 * c);
  double b1 = 13.0 / 12.0 * (b - 2.0 * c + d) * (b - 2.0 * c + d) +
              0.25 * (b - d) * (b - d);
  double b2 = 13.0 / 12.0 * (c - 2.0 * d + e) * (c - 2.0 * d + e) +
              0.25 * (3.0 * c - 4.0 * d + e) * (3.0 * c - 4.0 * d + e);
  double eps = 1e-6 * (a * a + b * b + c * c + d * d + e * e) / 5.0 + 1e-40;
  double a0 = 0.1 / ((eps + b0) * (eps + b0));
  double a1 = 0.6 / ((eps + b1) * (eps + b1));
  double a2 = 0.3 / ((eps + b2) * (eps + b2));
  return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
}

/* Slope limiters on undivided differences a = W_i - W_{i-1},
 * b = W_{i+1} - W_i. */
static double limit(int lim, double a, double b) {
  if (a * b <= 0.0) return 0.0;
  if (lim == LIM_MINMOD) return fabs(a) < fabs(b) ? a : b;
  /* monotonised central: sign(a) min(2|a|, 2|b|, |a+b|/2) */
  double m = 2.0 * fabs(a);
  if (2.0 * fabs(b) < m) m = 2.0 * fabs(b);
  if (0.5 * fabs(a + b) < m) m = 0.5 * fabs(a + b);
  return a > 0.0 ? m : -m;
}

/* HLLD flux (Miyoshi & Kusano 2005, J. Comput. Phys. 208, 315): the Riemann
 * fan is split by the outer fast waves S_L, S_R, the rotational waves
 * S*_L = S_M - |B_n|/sqrt(rho*_L), S*_R = S_M + |B_n|/sqrt(rho*_R) and the
 * contact S_M into four intermediate states with continuous normal velocity
 * (S_M) and total pressure (p_T*) across all of them, and density
 * continuous across the rotational waves.  The two face states share one
 * normal field, the mean of their B_n (a cell-centred scheme has a jump
 * there); the flux of B_n itself is the HLL value with the same outer
 * speeds, so its jump is still damped. */
static void hlld_flux(double gam, const double *wl0, const double *wr0, int n,
                      double *fs) {
  int t1 = n == 1 ? 2 : 1, t2 = n == 3 ? 2 : 3; /* tangential components */
  double bn = 0.5 * (wl0[4 + n] + wr0[4 + n]);
  double wl[NV], wr[NV], ul[NV], ur[NV], fl[NV], fr[NV];
  memcpy(wl, wl0, sizeof wl);
  memcpy(wr, wr0, sizeof wr);
  wl[4 + n] = bn;
  wr[4 + n] = bn;
  prim_to_cons(gam, wl, ul);
  prim_to_cons(gam, wr, ur);
  phys_flux(gam, wl, ul, n, fl);
  phys_flux(gam, wr, ur, n, fr);
  double cl = fast_speed(gam, wl, n), cr = fast_speed(gam, wr, n);
  double cmax = cl > cr ? cl : cr;
  double sl = (wl[n] < wr[n] ? wl[n] : wr[n]) - cmax;
  double sr = (wl[n] > wr[n] ? wl[n] : wr[n]) + cmax;
  /* HLL flux of the normal field (its physical flux is zero) */
  double fbn = 0.0;
  if (sl < 0.0 && sr > 0.0)
    fbn = sl * sr * (wr0[4 + n] - wl0[4 + n]) / (sr - sl);
  if (sl >= 0.0) {
    memcpy(fs, fl, sizeof fl);
    fs[4 + n] = fbn;
    return;
  }
  if (sr <= 0.0) {
    memcpy(fs, fr, sizeof fr);
    fs[4 + n] = fbn;
    return;
  }
  double ptl = wl[4] + 0.5 * (wl[5] * wl[5] + wl[6] * wl[6] + wl[7] * wl[7]);
  double ptr = wr[4] + 0.5 * (wr[5] * wr[5] + wr[6] * wr[6] + wr[7] * wr[7]);
  double dl = (sl - wl[n]) * wl[0], dr = (sr - wr[n]) * wr[0]; /* mass fluxes */
  double sm = (dr * wr[n] - dl * wl[n] - ptr + ptl) / (dr - dl);
  double pts = (dr * ptl - dl * ptr + dl * dr * (wr[n] - wl[n])) / (dr - dl);
  /* outer star states: U*_a from the jump conditions across S_a */
  double us[2][NV], rs[2];
  for (int a = 0; a < 2; ++a) {
    const double *w = a ? wr : wl, *u = a ? ur : ul;
    double s = a ? sr : sl, d = a ? dr : dl, pt = a ? ptr : ptl;
    double rho = d / (s - sm);
    double den = d * (s - sm) - bn * bn;
    double vt1, vt2, bt1, bt2;
    if (fabs(den) <= 1e-12 * (fabs(d * (s - sm)) + bn * bn)) {
      vt1 = w[t1]; vt2 = w[t2]; bt1 = w[4 + t1]; bt2 = w[4 + t2];
    } else {
      double fv = bn * (sm - w[n]) / den;
      double fb = (d * (s - w[n]) - bn * bn) / den;
      vt1 = w[t1] - w[4 + t1] * fv;
      vt2 = w[t2] - w[4 + t2] * fv;
      bt1 = w[4 + t1] * fb;
      bt2 = w[4 + t2] * fb;
    }
    double vb = w[1] * w[5] + w[2] * w[6] + w[3] * w[7];
    double vbs = sm * bn + vt1 * bt1 + vt2 * bt2;
    double e = ((s - w[n]) * u[4] - pt * w[n] + pts * sm + bn * (vb - vbs)) / (s - sm);
    double *q = us[a];
    q[0] = rho;
    q[n] = rho * sm;
    q[t1] = rho * vt1;
    q[t2] = rho * vt2;
    q[4] = e;
    q[4 + n] = bn;
    q[4 + t1] = bt1;
    q[4 + t2] = bt2;
    rs[a] = sqrt(rho);
  }
  double sgn = bn >= 0.0 ? 1.0 : -1.0;
  double ssl = sm - fabs(bn) / rs[0], ssr = sm + fabs(bn) / rs[1];
  /* F*_a = F_a + S_a (U*_a - U_a) */
  double fsl[NV], fsr[NV];
  for (int v = 0; v < NV; ++v) {
    fsl[v] = fl[v] + sl * (us[0][v] - ul[v]);
    fsr[v] = fr[v] + sr * (us[1][v] - ur[v]);
  }
  if (ssl >= 0.0 || ssr <= 0.0) {
    memcpy(fs, ssl >= 0.0 ? fsl : fsr, NV * sizeof(double));
    fs[4 + n] = fbn;
    return;
  }
  /* inner (double-star) states between the rotational waves */
  double vl1 = us[0][t1] / us[0][0], vl2 = us[0][t2] / us[0][0];
  double vr1 = us[1][t1] / us[1][0], vr2 = us[1][t2] / us[1][0];
  double sq = rs[0] + rs[1];
  double v1 = (rs[0] * vl1 + rs[1] * vr1 + (us[1][4 + t1] - us[0][4 + t1]) * sgn) / sq;
  double v2 = (rs[0] * vl2 + rs[1] * vr2 + (us[1][4 + t2] - us[0][4 + t2]) * sgn) / sq;
  double b1 = (rs[0] * us[1][4 + t1] + rs[1] * us[0][4 + t1] +
               rs[0] * rs[1] * (vr1 - vl1) * sgn) / sq;
  double b2 = (rs[0] * us[1][4 + t2] + rs[1] * us[0][4 + t2] +
               rs[0] * rs[1] * (vr2 - vl2) * sgn) / sq;
  double vbss = sm * bn + v1 * b1 + v2 * b2;
  int a = sm >= 0.0 ? 0 : 1;
  const double *q = us[a];
  double vbs = (q[n] * q[4 + n] + q[t1] * q[4 + t1] + q[t2] * q[4 + t2]) / q[0];
  double uss[NV];
  uss[0] = q[0];
  uss[n] = q[0] * sm;
  uss[t1] = q[0] * v1;
  uss[t2] = q[0] * v2;
  uss[4] = q[4] + (a ? 1.0 : -1.0) * rs[a] * (vbs - vbss) * sgn;
  uss[4 + n] = bn;
  uss[4 + t1] = b1;
  uss[4 + t2] = b2;
  /* F**_a = F*_a + S*_a (U**_a - U*_a) */
  double ssa = a ? ssr : ssl;
  const double *fa = a ? fsr : fsl;
  for (int v = 0; v < NV; ++v) fs[v] = fa[v] + ssa * (uss[v] - q[v]);
  fs[4 + n] = fbn;
}

/* Numerical flux through one face from left/right face states. */
static void face_flux(const orc_ctx *c, const double *wl, const double *wr,
                      int n, double *fs) {
  if (c->flux == FLUX_HLLD) {
    hlld_flux(c->gamma, wl, wr, n, fs);
    return;
  }
  double gam = c->gamma;
  double ul[NV], ur[NV], fl[NV], fr[NV];
  prim_to_cons(gam, wl, ul);
  prim_to_cons(gam, wr, ur);
  phys_flux(gam, wl, ul, n, fl);
  phys_flux(gam, wr, ur, n, fr);
  double cl = fast_speed(gam, wl, n), cr = fast_speed(gam, wr, n);
  if (c->flux == FLUX_TVDLF) {
    /* F* = (F_L + F_R)/2 - alpha (U_R - U_L)/2, alpha = max |v_n| + c_f */
    double al = fabs(wl[n]) + cl, ar = fabs(wr[n]) + cr;
    double alpha = al > ar ? al : ar;
    for (int v = 0; v < NV; ++v)
      fs[v] = 0.5 * (fl[v] + fr[v]) - 0.5 * alpha * (ur[v] - ul[v]);
  } else {
    /* HLL with S_L = min(v_nL - c_fL, v_nR - c_fR), S_R = max(...+...) */
    double sl = wl[n] - cl, sr = wr[n] + cr;
    if (wr[n] - cr < sl) sl = wr[n] - cr;
    if (wl[n] + cl > sr) sr = wl[n] + cl;
    if (sl >= 0.0) {
      for (int v = 0; v < NV; ++v) fs[v] = fl[v];
    } else if (sr <= 0.0) {
      for (int v = 0; v < NV; ++v) fs[v] = fr[v];
    } else {
      for (int v = 0; v < NV; ++v)
        fs[v] = (sr * fl[v] - sl * fr[v] + sl * sr * (ur[v] - ul[v])) /
                (sr - sl);
    }
  }
}

/* The numerical flux of this oracle's scheme for one face (test access):
 * primitive face states wl, wr (code units), normal component n = 1..3. */
int orc_ghosts(const void *h) { return ((const orc_ctx *)h)->ng; }

void orc_face_flux(void *h, const double *wl, const double *wr, int n, double *out) {
  face_flux((const orc_ctx *)h, wl, wr, n, out);
}

/* ---- grid ------------------------------------------------------------------ */
static void *xcalloc(size_t n, size_t s) {
  void *p = calloc(n, s);
  return p;
}

/* Spherical: geometric radial stretch r_{i-1/2} = r_in q^i with
 * q = (r_out/r_in)^(1/nr) (radially stretched grid, Sect. 2); uniform
 * colatitude and longitude.  Cell centres are arithmetic means of the two
 * edges.  Slab: uniform in all three directions. */
static void build_grid(orc_ctx *c, const double *dp) {
  c->re = xcalloc(c->nr + 1, sizeof(double));
  c->te = xcalloc(c->nt + 1, sizeof(double));
  c->pe = xcalloc(c->np + 1, sizeof(double));
  c->rc = xcalloc(c->nr, sizeof(double));
  c->tc = xcalloc(c->nt, sizeof(double));
  c->pc = xcalloc(c->np, sizeof(double));
  if (c->geom == GEOM_SPH) {
    double r0 = dp[0] / u_len(), r1 = dp[1] / u_len();
    double q = pow(r1 / r0, 1.0 / c->nr);
    for (int i = 0; i <= c->nr; ++i) c->re[i] = r0 * pow(q, (double)i);
    c->re[c->nr] = r1;
    double t0 = dp[2], t1 = dp[3];
    for (int j = 0; j <= c->nt; ++j)
      c->te[j] = t0 + (t1 - t0) * (double)j / c->nt;
    /* longitude range: the full circle (periodic), or a sub-range for a
     * block of a refined grid whose ghosts the caller sets */
    double p0 = dp[13], p1 = dp[14];
    for (int k = 0; k <= c->np; ++k)
      c->pe[k] = p0 + (p1 - p0) * (double)k / c->np;
  } else {
    double lo[3] = {dp[7], dp[9], dp[11]}, hi[3] = {dp[8], dp[10], dp[12]};
    for (int i = 0; i <= c->nr; ++i)
      c->re[i] = lo[0] + (hi[0] - lo[0]) * (double)i / c->nr;
    for (int j = 0; j <= c->nt; ++j)
      c->te[j] = lo[1] + (hi[1] - lo[1]) * (double)j / c->nt;
    for (int k = 0; k <= c->np; ++k)
      c->pe[k] = lo[2] + (hi[2] - lo[2]) * (double)k / c->np;
  }
  for (int i = 0; i < c->nr; ++i) c->rc[i] = 0.5 * (c->re[i] + c->re[i + 1]);
  for (int j = 0; j < c->nt; ++j) c->tc[j] = 0.5 * (c->te[j] + c->te[j + 1]);
  for (int k = 0; k < c->np; ++k) c->pc[k] = 0.5 * (c->pe[k] + c->pe[k + 1]);
}

/* Per-axis 1D factors of the spherical finite-volume metric: per r cell
 * (r+^3 - r-^3)/3, (r+^2 - r-^2)/V_r and half of it; per theta cell
 * cos t- - cos t+, (sin t+ - sin t-)/(cos t- - cos t+), sin and cos of the
 * centre; sin of every theta edge. */
static void build_metric(orc_ctx *c) {
  c->volr = xcalloc(c->nr, sizeof(double));
  c->hr = xcalloc(c->nr, sizeof(double));
  c->garea = xcalloc(c->nr, sizeof(double));
  c->ct = xcalloc(c->nt, sizeof(double));
  c->st = xcalloc(c->nt, sizeof(double));
  c->snc = xcalloc(c->nt, sizeof(double));
  c->csc = xcalloc(c->nt, sizeof(double));
  c->se = xcalloc(c->nt + 1, sizeof(double));
  for (int i = 0; i < c->nr; ++i) {
    double rm = c->re[i], rp = c->re[i + 1];
    c->volr[i] = (rp * rp * rp - rm * rm * rm) / 3.0;
    c->garea[i] = (rp * rp - rm * rm) / c->volr[i];
    c->hr[i] = (rp * rp - rm * rm) / (2.0 * c->volr[i]);
  }
  for (int j = 0; j <= c->nt; ++j) c->se[j] = sin(c->te[j]);
  for (int j = 0; j < c->nt; ++j) {
    c->ct[j] = cos(c->te[j]) - cos(c->te[j + 1]);
    c->st[j] = (c->se[j + 1] - c->se[j]) / c->ct[j];
    c->snc[j] = sin(c->tc[j]);
    c->csc[j] = cos(c->tc[j]);
  }
}

/* ip: nr nt np geom flux limiter gravity corot bc_transverse bc_mode slab_bcx
 *     tracer
 * dp: r_in[m] r_out[m] th_min th_max gamma omega[rad/s] cfl
 *     x0 x1 y0 y1 z0 z1 (slab only, code units) ph_min ph_max (spherical) */
void *orc_create(const int *ip, const double *dp) {
  orc_ctx *c = xcalloc(1, sizeof(orc_ctx));
  if (!c) return 0;
  c->nr = ip[0];
  c->nt = ip[1];
  c->np = ip[2];
  c->geom = ip[3];
  c->flux = ip[4];
  c->limiter = ip[5];
  c->gravity = ip[6];
  c->corot = ip[7];
  c->bc_transverse = ip[8];
  c->bc_mode = ip[9];
  c->slab_bcx = ip[10];
  c->tracer = ip[11] && ip[3] == GEOM_SPH;
  c->ng = c->limiter == LIM_WENO5 ? 3 : 2;
  /* asymm mirrors active cell g-1 into ghost layer g: needs ng cells in r */
  if (c->bc_transverse == BCT_ASYMM && c->nr < c->ng) {
    free(c);
    return 0;
  }
  c->gr = c->nr + 2 * c->ng;
  c->gt = c->nt + 2 * c->ng;
  c->gp = c->np + 2 * c->ng;
  c->gamma = dp[4];
  c->cfl = dp[6];
  if (c->geom == GEOM_SPH) {
    c->omega = c->corot ? dp[5] * u_time() : 0.0;
    c->gm = c->gravity ? GM_SUN / (u_len() * V_UNIT * V_UNIT) : 0.0;
  } else {
    c->omega = 0.0;
    c->gm = 0.0;
  }
  build_grid(c, dp);
  build_metric(c);
  size_t n = pad_cells(c) * NV;
  c->U = xcalloc(n, sizeof(double));
  c->U0 = xcalloc(n, sizeof(double));
  c->U1 = xcalloc(n, sizeof(double));
  c->W = xcalloc(n, sizeof(double));
  c->F = xcalloc(n, sizeof(double));
  c->L = xcalloc(n, sizeof(double));
  if (!c->U || !c->U0 || !c->U1 || !c->W || !c->F || !c->L) return 0;
  if (c->tracer) {
    size_t m = pad_cells(c);
    c->T = xcalloc(m, sizeof(double));
    c->T0 = xcalloc(m, sizeof(double));
    c->T1 = xcalloc(m, sizeof(double));
    c->LT = xcalloc(m, sizeof(double));
    c->P = xcalloc(m, sizeof(double));
    c->FT = xcalloc(m, sizeof(double));
    if (!c->T || !c->T0 || !c->T1 || !c->LT || !c->P || !c->FT) return 0;
  }
  return c;
}

void orc_destroy(void *h) {
  orc_ctx *c = h;
  if (!c) return;
  free(c->re); free(c->te); free(c->pe);
  free(c->rc); free(c->tc); free(c->pc);
  free(c->U); free(c->U0); free(c->U1);
  free(c->W); free(c->F); free(c->L);
  free(c->T); free(c->T0); free(c->T1); free(c->LT); free(c->P); free(c->FT);
  free(c->tau); free(c->maps); free(c->cme);
  free(c->volr); free(c->hr); free(c->garea); free(c->ct);
  free(c->st); free(c->snc); free(c->csc); free(c->se);
  free(c);
}

/* Units for callers: t, length, rho, p, B, velocity. */
void orc_units(double *out) {
  out[0] = u_time();
  out[1] = u_len();
  out[2] = u_rho();
  out[3] = u_pres();
  out[4] = u_bfield();
  out[5] = V_UNIT;
}

/* Grid edges (code units, angles in radians). */
void orc_edges(const void *h, double *r, double *t, double *p) {
  const orc_ctx *c = h;
  memcpy(r, c->re, sizeof(double) * (c->nr + 1));
  memcpy(t, c->te, sizeof(double) * (c->nt + 1));
  memcpy(p, c->pe, sizeof(double) * (c->np + 1));
}

/* ---- boundary data ----------------------------------------------------------- */

/* Maps: primitive SI, [n][8][nt][np]: rho, v_r, v_t, v_p (co-rotating), p,
 * B_r, B_t, B_p.  Times in seconds, strictly ascending. */
int orc_set_maps(void *h, int n, const double *t_s, const double *maps_si) {
  orc_ctx *c = h;
  if (n < 1) return -1;
  for (int m = 1; m < n; ++m)
    if (!(t_s[m] > t_s[m - 1])) return -1;
  free(c->tau);
  free(c->maps);
  c->n_maps = n;
  c->tau = xcalloc(n, sizeof(double));
  size_t plane = (size_t)c->nt * c->np;
  c->maps = xcalloc((size_t)n * NV * plane, sizeof(double));
  double scale[NV] = {u_rho(), V_UNIT, V_UNIT, V_UNIT, u_pres(),
                      u_bfield(), u_bfield(), u_bfield()};
  for (int m = 0; m < n; ++m) {
    c->tau[m] = t_s[m] / u_time();
    for (int v = 0; v < NV; ++v)
      for (size_t q = 0; q < plane; ++q) {
        size_t o = ((size_t)m * NV + v) * plane + q;
        c->maps[o] = maps_si[o] / scale[v];
      }
  }
  for (size_t o = 0; o < (size_t)n * plane; ++o) {
    size_t m = o / plane, q = o % plane;
    if (!(c->maps[(m * NV + 0) * plane + q] > 0.0)) return -2;
    if (!(c->maps[(m * NV + 4) * plane + q] > 0.0)) return -2;
  }
  return 0;
}

/* Cone CMEs, SI rows of 8: t_start[s], duration[s], latitude[rad],
 * longitude (co-rotating)[rad], half-width[rad], speed[m/s],
 * density[kg/m^3], temperature[K]. */
int orc_set_cmes(void *h, int n, const double *rows) {
  orc_ctx *c = h;
  free(c->cme);
  c->cme = 0;
  c->n_cme = n;
  if (n <= 0) {
    c->n_cme = 0;
    return 0;
  }
  c->cme = xcalloc((size_t)n * 8, sizeof(double));
  for (int q = 0; q < n; ++q) {
    const double *s = rows + 8 * q;
    double *d = c->cme + 8 * q;
    d[0] = s[0] / u_time();
    d[1] = s[1] / u_time();
    d[2] = 0.5 * 3.14159265358979323846 - s[2]; /* colatitude */
    d[3] = s[3];
    d[4] = s[4];
    d[5] = s[5] / V_UNIT;
    d[6] = s[6] / u_rho();
    /* fully ionised hydrogen: p = 2 n k_B T with n = rho / m_p */
    d[7] = 2.0 * (s[6] / M_PROTON) * K_BOLTZ * s[7] / u_pres();
  }
  return 0;
}

/* Linear interpolation in time between the two maps that bracket t, clamped
 * to the first/last map outside their range (Sect. 3). */
static void map_at(const orc_ctx *c, double t, int j, int k, double *w) {
  size_t plane = (size_t)c->nt * c->np, q = (size_t)j * c->np + k;
  int n = c->n_maps;
  if (n == 1 || t <= c->tau[0]) {
    for (int v = 0; v < NV; ++v) w[v] = c->maps[(size_t)v * plane + q];
    return;
  }
  if (t >= c->tau[n - 1]) {
    for (int v = 0; v < NV; ++v)
      w[v] = c->maps[((size_t)(n - 1) * NV + v) * plane + q];
    return;
  }
  int m = 0;
  while (m + 1 < n - 1 && c->tau[m + 1] <= t) ++m;
  double wgt = (t - c->tau[m]) / (c->tau[m + 1] - c->tau[m]);
  for (int v = 0; v < NV; ++v) {
    double a = c->maps[((size_t)m * NV + v) * plane + q];
    double b = c->maps[((size_t)(m + 1) * NV + v) * plane + q];
    w[v] = (1.0 - wgt) * a + wgt * b;
  }
}

/* Boundary primitive at the inner shell for cell column (j, k) at time t:
 * the time-interpolated map, then the cone-CME overwrite of points whose
 * great-circle distance to the cone axis is within the half-width while the
 * CME is being inserted (Sect. 3.2).  The CME is not magnetised: B is kept. */
/* 1 when boundary point (j, k) lies inside a cone CME being inserted at t */
static int in_cme(const orc_ctx *c, double t, int j, int k, int q) {
  const double *m = c->cme + 8 * q;
  if (!(t >= m[0] && t < m[0] + m[1])) return 0;
  double th = c->tc[j], ph = c->pc[k];
  double cosd = cos(th) * cos(m[2]) + sin(th) * sin(m[2]) * cos(ph - m[3]);
  return cosd >= cos(m[4]);
}

static void inner_boundary_prim(const orc_ctx *c, double t, int j, int k,
                                double *w) {
  map_at(c, t, j, k, w);
  double th = c->tc[j];
  for (int q = 0; q < c->n_cme; ++q) {
    const double *m = c->cme + 8 * q;
    if (in_cme(c, t, j, k, q)) {
      w[0] = m[6];
      w[1] = m[5];
      w[2] = 0.0;
      w[3] = -c->omega * c->re[0] * sin(th);
      w[4] = m[7];
    }
  }
}

/* Fill the two ghost layers on every side of U at time t. */
static void fill_ghosts(orc_ctx *c, double *U, double t) {
  if (c->bc_mode == BCM_FROZEN) return;
  int nr = c->nr, nt = c->nt, np = c->np;
  if (c->geom == GEOM_SPH) {
    /* inner radial boundary from the maps: the same value in both layers */
    for (int k = 0; k < np; ++k)
      for (int j = 0; j < nt; ++j) {
        double w[NV], u[NV];
        inner_boundary_prim(c, t, j, k, w);
        for (int g = 1; g <= c->ng; ++g) {
          double wg[NV];
          memcpy(wg, w, sizeof wg);
          if (c->bc_transverse == BCT_ASYMM) {
            /* transverse components vanish on the boundary surface:
             * ghost = minus the mirror-image active cell (primitive) */
            double um[NV], wm[NV];
            for (int v = 0; v < NV; ++v) um[v] = U[IX(c, v, g - 1, j, k)];
            cons_to_prim(c->gamma, um, wm);
            wg[2] = -wm[2];
            wg[3] = -wm[3];
            wg[6] = -wm[6];
            wg[7] = -wm[7];
          }
          prim_to_cons(c->gamma, wg, u);
          for (int v = 0; v < NV; ++v) U[IX(c, v, -g, j, k)] = u[v];
        }
      }
    /* outer radial boundary: zero-gradient outflow */
    for (int v = 0; v < NV; ++v)
      for (int k = 0; k < np; ++k)
        for (int j = 0; j < nt; ++j)
          for (int g = 0; g < c->ng; ++g)
            U[IX(c, v, nr + g, j, k)] = U[IX(c, v, nr - 1, j, k)];
    /* colatitude edges: reflecting.  Ghost layer g mirrors active row g-1
     * from the edge (the last row when the grid has fewer rows) with the
     * theta components of momentum and field negated, so that no mass,
     * magnetic flux or energy crosses the edge. */
    for (int v = 0; v < NV; ++v) {
      double sgn = (v == 2 || v == 6) ? -1.0 : 1.0;
      for (int k = 0; k < np; ++k)
        for (int i = 0; i < nr; ++i)
          for (int g = 1; g <= c->ng; ++g) {
            int lo = g - 1 < nt ? g - 1 : nt - 1;
            int hi = nt - g >= 0 ? nt - g : 0;
            U[IX(c, v, i, -g, k)] = sgn * U[IX(c, v, i, lo, k)];
            U[IX(c, v, i, nt - 1 + g, k)] = sgn * U[IX(c, v, i, hi, k)];
          }
    }
  } else {
    for (int v = 0; v < NV; ++v)
      for (int k = 0; k < np; ++k)
        for (int j = 0; j < nt; ++j)
          for (int g = 1; g <= c->ng; ++g) {
            if (c->slab_bcx == SLABX_PERIODIC) {
              U[IX(c, v, -g, j, k)] = U[IX(c, v, nr - g, j, k)];
              U[IX(c, v, nr - 1 + g, j, k)] = U[IX(c, v, g - 1, j, k)];
            } else {
              U[IX(c, v, -g, j, k)] = U[IX(c, v, 0, j, k)];
              U[IX(c, v, nr - 1 + g, j, k)] = U[IX(c, v, nr - 1, j, k)];
            }
          }
    for (int v = 0; v < NV; ++v)
      for (int k = 0; k < np; ++k)
        for (int i = 0; i < nr; ++i)
          for (int g = 1; g <= c->ng; ++g) {
            U[IX(c, v, i, -g, k)] = U[IX(c, v, i, nt - g, k)];
            U[IX(c, v, i, nt - 1 + g, k)] = U[IX(c, v, i, g - 1, k)];
          }
  }
  /* longitude: periodic (slab z: periodic) */
  for (int v = 0; v < NV; ++v)
    for (int g = 1; g <= c->ng; ++g)
      for (int j = -c->ng; j < nt + c->ng; ++j)
        for (int i = -c->ng; i < nr + c->ng; ++i) {
          U[IX(c, v, i, j, -g)] = U[IX(c, v, i, j, np - g)];
          U[IX(c, v, i, j, np - 1 + g)] = U[IX(c, v, i, j, g - 1)];
        }
}

/* ---- metric -------------------------------------------------------------- */
/* Per-cell geometric factors of the finite-volume divergence.  Spherical
 * volume V = (r+^3 - r-^3)/3 (cos t- - cos t+) dphi, r-face area r^2 (cos t-
 * - cos t+) dphi, theta-face area sin t (r+^2 - r-^2)/2 dphi, phi-face area
 * (r+^2 - r-^2)/2 dtheta. */

/* ---- one evaluation of dU/dt = L(U) over active cells --------------------- */
/* Upwind tracer values tau = (rho tau) / rho of every active cell, and of the
 * ghost cells: inside an inserted CME cone 1, elsewhere 0 at the inner
 * boundary; the edge cell's value beyond r_out and the colatitude edges;
 * periodic in phi. */
static void tracer_upwind(orc_ctx *c, const double *U, const double *T, double t) {
  int nr = c->nr, nt = c->nt, np = c->np;
  if (c->bc_mode == BCM_FROZEN) { /* ghosts set by the caller: tau = T / rho */
    size_t n = pad_cells(c);
    for (size_t o = 0; o < n; ++o) c->P[o] = U[o] != 0.0 ? T[o] / U[o] : 0.0;
    return;
  }
  for (int k = 0; k < np; ++k)
    for (int j = 0; j < nt; ++j)
      for (int i = 0; i < nr; ++i)
        c->P[IX(c, 0, i, j, k)] = T[IX(c, 0, i, j, k)] / U[IX(c, 0, i, j, k)];
  for (int k = 0; k < np; ++k)
    for (int j = 0; j < nt; ++j) {
      double ind = 0.0;
      for (int q = 0; q < c->n_cme; ++q)
        if (in_cme(c, t, j, k, q)) ind = 1.0;
      for (int g = 1; g <= c->ng; ++g) {
        c->P[IX(c, 0, -g, j, k)] = ind;
        c->P[IX(c, 0, nr - 1 + g, j, k)] = c->P[IX(c, 0, nr - 1, j, k)];
      }
    }
  for (int k = 0; k < np; ++k)
    for (int i = 0; i < nr; ++i)
      for (int g = 1; g <= c->ng; ++g) {
        c->P[IX(c, 0, i, -g, k)] = c->P[IX(c, 0, i, 0, k)];
        c->P[IX(c, 0, i, nt - 1 + g, k)] = c->P[IX(c, 0, i, nt - 1, k)];
      }
  for (int j = 0; j < nt; ++j)
    for (int i = 0; i < nr; ++i)
      for (int g = 1; g <= c->ng; ++g) {
        c->P[IX(c, 0, i, j, -g)] = c->P[IX(c, 0, i, j, np - g)];
        c->P[IX(c, 0, i, j, np - 1 + g)] = c->P[IX(c, 0, i, j, g - 1)];
      }
}

/* Right-hand side L = -div F + S of every active cell (and, with the tracer
 * on, LT = -div(F_rho tau_upwind) from the same mass fluxes). */
/* bf (may be NULL): the face fluxes on the six faces of the active box,
 * [9][...] per face (the 8 variables and the tracer flux), faces in the
 * order r-low, r-high ([np][nt] each), theta-low, theta-high ([np][nr]),
 * phi-low, phi-high ([nt][nr]). */
static void compute_rhs_bf(orc_ctx *c, double *U, double *L, double *bnd,
                           const double *T, double *LT, double *tbnd, double t,
                           double *bf);
static void compute_rhs(orc_ctx *c, double *U, double *L, double *bnd,
                        const double *T, double *LT, double *tbnd, double t) {
  compute_rhs_bf(c, U, L, bnd, T, LT, tbnd, t, 0);
}

static void compute_rhs_bf(orc_ctx *c, double *U, double *L, double *bnd,
                           const double *T, double *LT, double *tbnd, double t,
                           double *bf) {
  int nr = c->nr, nt = c->nt, np = c->np;
  double gam = c->gamma;
  size_t np_cells = pad_cells(c);
  double *W = c->W, *F = c->F;
  if (T) {
    tracer_upwind(c, U, T, t);
    for (size_t o = 0; o < np_cells; ++o) LT[o] = 0.0;
    *tbnd = 0.0;
  }
  /* primitives of every padded cell whose ghosts were filled */
#pragma omp parallel for
  for (long q = 0; q < (long)np_cells; ++q) {
    double u[NV], w[NV];
    for (int v = 0; v < NV; ++v) u[v] = U[(size_t)v * np_cells + q];
    if (u[0] == 0.0) { /* unfilled corner ghost: never read */
      for (int v = 0; v < NV; ++v) W[(size_t)v * np_cells + q] = 0.0;
      continue;
    }
    cons_to_prim(gam, u, w);
    for (int v = 0; v < NV; ++v) W[(size_t)v * np_cells + q] = w[v];
  }
  for (size_t o = 0; o < np_cells * NV; ++o) L[o] = 0.0;
  for (int v = 0; v < NV; ++v) bnd[v] = 0.0;

  double dth = c->te[1] - c->te[0], dph = c->pe[1] - c->pe[0];

  /* three sweeps; face m-1/2 lies between cells m-1 and m, m = 0..n */
  for (int dir = 0; dir < 3; ++dir) {
    int n = dir == 0 ? nr : (dir == 1 ? nt : np);
    int di = dir == 0, dj = dir == 1, dk = dir == 2;
    int ei = nr + di, ej = nt + dj, ek = np + dk; /* face counts */
#pragma omp parallel for
    for (int k = 0; k < ek; ++k)
      for (int j = 0; j < ej; ++j)
        for (int i = 0; i < ei; ++i) {
          double wm2[NV], wm1[NV], w0[NV], wp1[NV], wl[NV], wr[NV], fs[NV];
          for (int v = 0; v < NV; ++v) {
            wm2[v] = W[IX(c, v, i - 2 * di, j - 2 * dj, k - 2 * dk)];
            wm1[v] = W[IX(c, v, i - di, j - dj, k - dk)];
            w0[v] = W[IX(c, v, i, j, k)];
            wp1[v] = W[IX(c, v, i + di, j + dj, k + dk)];
          }
          if (c->limiter == LIM_WENO5) {
            /* face m-1/2 from cells m-3 .. m+2; a face state with rho or p
             * <= 0 falls back to its cell value (first order) */
            double wm3[NV], wp2[NV];
            for (int v = 0; v < NV; ++v) {
              wm3[v] = W[IX(c, v, i - 3 * di, j - 3 * dj, k - 3 * dk)];
              wp2[v] = W[IX(c, v, i + 2 * di, j + 2 * dj, k + 2 * dk)];
            }
            for (int v = 0; v < NV; ++v) {
              wl[v] = weno5(wm3[v], wm2[v], wm1[v], w0[v], wp1[v]);
              wr[v] = weno5(wp2[v], wp1[v], w0[v], wm1[v], wm2[v]);
            }
            if (!(wl[0] > 0.0 && wl[4] > 0.0)) memcpy(wl, wm1, sizeof wl);
            if (!(wr[0] > 0.0 && wr[4] > 0.0)) memcpy(wr, w0, sizeof wr);
          } else {
            for (int v = 0; v < NV; ++v) {
              double sl = limit(c->limiter, wm1[v] - wm2[v], w0[v] - wm1[v]);
              double sr = limit(c->limiter, w0[v] - wm1[v], wp1[v] - w0[v]);
              wl[v] = wm1[v] + 0.5 * sl;
              wr[v] = w0[v] - 0.5 * sr;
            }
          }
          face_flux(c, wl, wr, dir + 1, fs);
          for (int v = 0; v < NV; ++v) F[IX(c, v, i, j, k)] = fs[v];
        }
    (void)n;
    /* tracer face flux: mass flux times tau of the upwind cell */
    if (T) {
#pragma omp parallel for
      for (int k = 0; k < ek; ++k)
        for (int j = 0; j < ej; ++j)
          for (int i = 0; i < ei; ++i) {
            double fm = F[IX(c, 0, i, j, k)];
            double up = fm >= 0.0 ? c->P[IX(c, 0, i - di, j - dj, k - dk)]
                                  : c->P[IX(c, 0, i, j, k)];
            c->FT[IX(c, 0, i, j, k)] = fm * up;
          }
    }
    /* the fluxes through the low and high faces of the active box */
    if (bf) {
      size_t off = 0, fsz[3];
      fsz[0] = (size_t)np * nt;
      fsz[1] = (size_t)np * nr;
      fsz[2] = (size_t)nt * nr;
      for (int d = 0; d < dir; ++d) off += 2 * 9 * fsz[d];
      for (int side = 0; side < 2; ++side)
        for (int v = 0; v < 9; ++v) {
          double *out = bf + off + ((size_t)side * 9 + v) * fsz[dir];
          size_t q = 0;
          int m = side ? n : 0;
          for (int a = 0; a < (dir == 2 ? nt : np); ++a)
            for (int b = 0; b < (dir == 0 ? nt : nr); ++b, ++q) {
              int i = dir == 0 ? m : b, j = dir == 0 ? b : (dir == 1 ? m : a);
              int k = dir == 2 ? m : a;
              out[q] = v < 8 ? F[IX(c, v, i, j, k)] : (T ? c->FT[IX(c, 0, i, j, k)] : 0.0);
            }
        }
    }
    /* divergence of the face fluxes, face m-1/2 stored at index m */
#pragma omp parallel for
    for (int k = 0; k < np; ++k)
      for (int j = 0; j < nt; ++j)
        for (int i = 0; i < nr; ++i) {
          for (int v = 0; v < NV; ++v) {
            double fm = F[IX(c, v, i, j, k)];
            double fp = F[IX(c, v, i + di, j + dj, k + dk)];
            double div;
            if (c->geom == GEOM_SLAB) {
              double h = dir == 0 ? c->re[1] - c->re[0]
                                  : (dir == 1 ? dth : dph);
              div = (fp - fm) / h;
            } else if (dir == 0) {
              double rm = c->re[i], rp = c->re[i + 1];
              div = (rp * rp * fp - rm * rm * fm) / c->volr[i];
            } else if (dir == 1) {
              div = c->hr[i] * (c->se[j + 1] * fp - c->se[j] * fm) / c->ct[j];
            } else {
              div = c->hr[i] * dth / (c->ct[j] * dph) * (fp - fm);
            }
            L[IX(c, v, i, j, k)] -= div;
          }
          if (T) {
            double fm = c->FT[IX(c, 0, i, j, k)];
            double fp = c->FT[IX(c, 0, i + di, j + dj, k + dk)];
            double div;
            if (dir == 0) {
              double rm = c->re[i], rp = c->re[i + 1];
              div = (rp * rp * fp - rm * rm * fm) / c->volr[i];
            } else if (dir == 1) {
              div = c->hr[i] * (c->se[j + 1] * fp - c->se[j] * fm) / c->ct[j];
            } else {
              div = c->hr[i] * dth / (c->ct[j] * dph) * (fp - fm);
            }
            LT[IX(c, 0, i, j, k)] -= div;
          }
        }
    /* boundary-face integrals (area * flux) of this sweep, for the
     * conservation budget; periodic directions are skipped (they cancel) */
    int periodic = dir == 2 || (c->geom == GEOM_SLAB && dir == 1) ||
                   (c->geom == GEOM_SLAB && dir == 0 &&
                    c->slab_bcx == SLABX_PERIODIC);
    if (!periodic)
      for (int v = 0; v < NV; ++v) {
        double s = 0.0;
        for (int k = 0; k < np; ++k)
          for (int j = 0; j < (dir == 1 ? 1 : nt); ++j)
            for (int i = 0; i < (dir == 0 ? 1 : nr); ++i) {
              /* low face at index (i,j,k), high face n cells further */
              int ih = i + di * nr, jh = j + dj * nt;
              double am, ap;
              if (c->geom == GEOM_SLAB) {
                am = ap = dth * dph; /* only x reaches here */
              } else if (dir == 0) {
                double r0 = c->re[0], r1 = c->re[nr];
                am = r0 * r0 * c->ct[j] * dph;
                ap = r1 * r1 * c->ct[j] * dph;
              } else {
                double rm = c->re[i], rp = c->re[i + 1];
                am = c->se[0] * 0.5 * (rp * rp - rm * rm) * dph;
                ap = c->se[nt] * 0.5 * (rp * rp - rm * rm) * dph;
              }
              s += ap * F[IX(c, v, ih, jh, k)] - am * F[IX(c, v, i, j, k)];
            }
        bnd[v] += s;
      }
    if (!periodic && T && c->geom == GEOM_SPH) {
      double s = 0.0;
      for (int k = 0; k < np; ++k)
        for (int j = 0; j < (dir == 1 ? 1 : nt); ++j)
          for (int i = 0; i < (dir == 0 ? 1 : nr); ++i) {
            int ih = i + di * nr, jh = j + dj * nt;
            double am, ap;
            if (dir == 0) {
              double r0 = c->re[0], r1 = c->re[nr];
              am = r0 * r0 * c->ct[j] * dph;
              ap = r1 * r1 * c->ct[j] * dph;
            } else {
              double rm = c->re[i], rp = c->re[i + 1];
              am = c->se[0] * 0.5 * (rp * rp - rm * rm) * dph;
              ap = c->se[nt] * 0.5 * (rp * rp - rm * rm) * dph;
            }
            s += ap * c->FT[IX(c, 0, ih, jh, k)] - am * c->FT[IX(c, 0, i, j, k)];
          }
      *tbnd += s;
    }
  }

  /* source terms at cell centres */
  if (c->geom == GEOM_SLAB) return;
#pragma omp parallel for
  for (int k = 0; k < np; ++k)
    for (int j = 0; j < nt; ++j)
      for (int i = 0; i < nr; ++i) {
        double w[NV];
        for (int v = 0; v < NV; ++v) w[v] = W[IX(c, v, i, j, k)];
        double rho = w[0], vr = w[1], vt = w[2], vp = w[3], p = w[4];
        double br = w[5], bt = w[6], bp = w[7];
        double r = c->rc[i];
        double sn = c->snc[j], cs = c->csc[j], cot = cs / sn;
        double gr = c->garea[i], hr = c->hr[i], st = c->st[j];
        double ptot = p + 0.5 * (br * br + bt * bt + bp * bp);
        double s[NV] = {0};
        /* geometric terms of the spherical divergence */
        s[1] = (rho * (vt * vt + vp * vp) - (bt * bt + bp * bp)) / r +
               ptot * gr;
        s[2] = (-(rho * vr * vt - br * bt) + cot * (rho * vp * vp - bp * bp)) /
                   r +
               ptot * hr * st;
        s[3] = -((rho * vp * vr - bp * br) + cot * (rho * vp * vt - bp * bt)) /
               r;
        s[6] = (vr * bt - vt * br) / r;
        s[7] = ((vr * bp - vp * br) + cot * (vt * bp - vp * bt)) / r;
        /* gravity g = -GM/r^2 e_r: momentum rho g, energy rho v.g */
        if (c->gravity) {
          double g = -c->gm / (r * r);
          s[1] += rho * g;
          s[4] += rho * vr * g;
        }
        /* co-rotating frame, Omega along the polar axis:
         * F = rho (Omega x r) x Omega + 2 rho v x Omega, energy v.F */
        if (c->corot) {
          double om = c->omega;
          s[1] += rho * om * om * r * sn * sn + 2.0 * rho * om * vp * sn;
          s[2] += rho * om * om * r * sn * cs + 2.0 * rho * om * vp * cs;
          s[3] += -2.0 * rho * om * (vr * sn + vt * cs);
          s[4] += rho * om * om * r * sn * (vr * sn + vt * cs);
        }
        for (int v = 0; v < NV; ++v) L[IX(c, v, i, j, k)] += s[v];
      }
}

/* ---- CFL ---------------------------------------------------------------- */
/* dt = CFL / max over active cells of sum_d (|v_d| + c_f,d) / dx_d with
 * dx_r = dr, dx_t = r dtheta, dx_p = r sin(theta) dphi (slab: dx, dy, dz). */
static double cfl_dt(const orc_ctx *c, const double *U) {
  double lmax = 0.0;
  double dth = c->te[1] - c->te[0], dph = c->pe[1] - c->pe[0];
#pragma omp parallel for reduction(max : lmax)
  for (int k = 0; k < c->np; ++k)
    for (int j = 0; j < c->nt; ++j)
      for (int i = 0; i < c->nr; ++i) {
        double u[NV], w[NV];
        for (int v = 0; v < NV; ++v) u[v] = U[IX(c, v, i, j, k)];
        cons_to_prim(c->gamma, u, w);
        double dx[3];
        dx[0] = c->re[i + 1] - c->re[i];
        if (c->geom == GEOM_SPH) {
          dx[1] = c->rc[i] * dth;
          dx[2] = c->rc[i] * sin(c->tc[j]) * dph;
        } else {
          dx[1] = dth;
          dx[2] = dph;
        }
        double lam = 0.0;
        for (int d = 0; d < 3; ++d)
          lam += (fabs(w[d + 1]) + fast_speed(c->gamma, w, d + 1)) / dx[d];
        if (lam > lmax) lmax = lam; /* invalid (NaN) cells are skipped; the
                                       step's validity check reports them */
      }
  return c->cfl / lmax;
}

double orc_dt(void *h) {
  orc_ctx *c = h;
  return cfl_dt(c, c->U) * u_time();
}

/* ---- one SSP-RK2 step ----------------------------------------------------- */
/* U1 = Un + dt L(Un) with ghosts at t; U^{n+1} = Un/2 + (U1 + dt L(U1))/2
 * with ghosts at t + dt.  Returns 0 or the index+1 of the first cell with
 * rho <= 0, p <= 0 or a non-finite value (negated). */
static long rk2_step(orc_ctx *c, double dt) {
  size_t n = pad_cells(c) * NV;
  int nr = c->nr, nt = c->nt, np = c->np;
  double b1[NV], b2[NV];
  size_t nt1 = pad_cells(c);
  double tb1 = 0.0, tb2 = 0.0;
  memcpy(c->U0, c->U, n * sizeof(double));
  if (c->tracer) memcpy(c->T0, c->T, nt1 * sizeof(double));
  fill_ghosts(c, c->U0, c->t);
  compute_rhs(c, c->U0, c->L, b1, c->tracer ? c->T0 : 0, c->LT, &tb1, c->t);
  if (c->tracer) {
    memcpy(c->T1, c->T0, nt1 * sizeof(double));
    for (int k = 0; k < np; ++k)
      for (int j = 0; j < nt; ++j)
        for (int i = 0; i < nr; ++i) {
          size_t o = IX(c, 0, i, j, k);
          c->T1[o] = c->T0[o] + dt * c->LT[o];
        }
  }
  memcpy(c->U1, c->U0, n * sizeof(double));
#pragma omp parallel for
  for (int k = 0; k < np; ++k)
    for (int j = 0; j < nt; ++j)
      for (int i = 0; i < nr; ++i)
        for (int v = 0; v < NV; ++v) {
          size_t o = IX(c, v, i, j, k);
          c->U1[o] = c->U0[o] + dt * c->L[o];
        }
  fill_ghosts(c, c->U1, c->t + dt);
  compute_rhs(c, c->U1, c->L, b2, c->tracer ? c->T1 : 0, c->LT, &tb2, c->t + dt);
  if (c->tracer) {
    for (int k = 0; k < np; ++k)
      for (int j = 0; j < nt; ++j)
        for (int i = 0; i < nr; ++i) {
          size_t o = IX(c, 0, i, j, k);
          c->T[o] = 0.5 * c->T0[o] + 0.5 * (c->T1[o] + dt * c->LT[o]);
        }
    c->tbflux = 0.5 * dt * (tb1 + tb2);
  }
#pragma omp parallel for
  for (int k = 0; k < np; ++k)
    for (int j = 0; j < nt; ++j)
      for (int i = 0; i < nr; ++i)
        for (int v = 0; v < NV; ++v) {
          size_t o = IX(c, v, i, j, k);
          c->U[o] = 0.5 * c->U0[o] + 0.5 * (c->U1[o] + dt * c->L[o]);
        }
  for (int v = 0; v < NV; ++v) c->bflux[v] = 0.5 * dt * (b1[v] + b2[v]);
  /* residual ||rho^{n+1} - rho^n|| / ||rho^n||, fixed summation order */
  double s1 = 0.0, s0 = 0.0;
  for (int k = 0; k < np; ++k)
    for (int j = 0; j < nt; ++j)
      for (int i = 0; i < nr; ++i) {
        size_t o = IX(c, 0, i, j, k);
        double d = c->U[o] - c->U0[o];
        s1 += d * d;
        s0 += c->U0[o] * c->U0[o];
      }
  c->last_resid = sqrt(s1) / sqrt(s0);
  /* validity check */
  for (int k = 0; k < np; ++k)
    for (int j = 0; j < nt; ++j)
      for (int i = 0; i < nr; ++i) {
        double u[NV], w[NV];
        int bad = 0;
        for (int v = 0; v < NV; ++v) {
          u[v] = c->U[IX(c, v, i, j, k)];
          if (!isfinite(u[v])) bad = 1;
        }
        if (!bad) {
          cons_to_prim(c->gamma, u, w);
          if (!(w[0] > 0.0) || !(w[4] > 0.0)) bad = 1;
        }
        if (bad) return 1 + ((long)k * nt + j) * nr + i;
      }
  return 0;
}

/* Advance n steps (stop at t_end_s if > 0).  info: steps taken, t [s],
 * last dt [s], last residual, status (0 ok, -3 non-physical), bad cell. */
int orc_step(void *h, int n, double t_end_s, double *info) {
  orc_ctx *c = h;
  double tend = t_end_s > 0.0 ? t_end_s / u_time() : -1.0;
  int taken = 0;
  long bad = 0;
  for (int s = 0; s < n; ++s) {
    if (tend > 0.0 && c->t >= tend) break;
    double dt = cfl_dt(c, c->U);
    int clip = 0;
    if (tend > 0.0 && c->t + dt >= tend) {
      dt = tend - c->t;
      clip = 1;
    }
    bad = rk2_step(c, dt);
    c->t = clip ? tend : c->t + dt;
    c->step += 1;
    c->last_dt = dt;
    ++taken;
    if (bad) break;
  }
  if (info) {
    info[0] = taken;
    info[1] = c->t * u_time();
    info[2] = c->last_dt * u_time();
    info[3] = c->last_resid;
    info[4] = bad ? -3 : 0;
    info[5] = bad ? (double)(bad - 1) : -1.0;
  }
  return bad ? -3 : 0;
}

/* ---- state I/O -------------------------------------------------------------- */
/* kind 0: primitive SI, active [8][np][nt][nr]; 1: conservative code,
 * active; 2: conservative code, padded with ghosts; 3: primitive code,
 * active. */
int orc_set_state(void *h, const double *in, int kind) {
  orc_ctx *c = h;
  int nr = c->nr, nt = c->nt, np = c->np;
  if (kind == 2) {
    memcpy(c->U, in, pad_cells(c) * NV * sizeof(double));
    return 0;
  }
  double scale[NV] = {u_rho(), V_UNIT, V_UNIT, V_UNIT, u_pres(),
                      u_bfield(), u_bfield(), u_bfield()};
  size_t act = (size_t)nr * nt * np;
  for (int k = 0; k < np; ++k)
    for (int j = 0; j < nt; ++j)
      for (int i = 0; i < nr; ++i) {
        size_t q = ((size_t)k * nt + j) * nr + i;
        double a[NV], u[NV];
        for (int v = 0; v < NV; ++v) a[v] = in[v * act + q];
        if (kind == 0)
          for (int v = 0; v < NV; ++v) a[v] /= scale[v];
        if (kind == 1)
          memcpy(u, a, sizeof u);
        else
          prim_to_cons(c->gamma, a, u);
        for (int v = 0; v < NV; ++v) c->U[IX(c, v, i, j, k)] = u[v];
      }
  if (c->tracer) memset(c->T, 0, pad_cells(c) * sizeof(double));
  return 0;
}

int orc_get_state(void *h, double *out, int kind) {
  orc_ctx *c = h;
  int nr = c->nr, nt = c->nt, np = c->np;
  if (kind == 2) {
    memcpy(out, c->U, pad_cells(c) * NV * sizeof(double));
    return 0;
  }
  double scale[NV] = {u_rho(), V_UNIT, V_UNIT, V_UNIT, u_pres(),
                      u_bfield(), u_bfield(), u_bfield()};
  size_t act = (size_t)nr * nt * np;
  for (int k = 0; k < np; ++k)
    for (int j = 0; j < nt; ++j)
      for (int i = 0; i < nr; ++i) {
        size_t q = ((size_t)k * nt + j) * nr + i;
        double u[NV], w[NV];
        for (int v = 0; v < NV; ++v) u[v] = c->U[IX(c, v, i, j, k)];
        if (kind == 1) {
          for (int v = 0; v < NV; ++v) out[v * act + q] = u[v];
          continue;
        }
        cons_to_prim(c->gamma, u, w);
        if (kind == 0)
          for (int v = 0; v < NV; ++v) w[v] *= scale[v];
        for (int v = 0; v < NV; ++v) out[v * act + q] = w[v];
      }
  return 0;
}

/* Ghost layers as seen by the update at time t_s: fills the padded state and
 * returns it (kind 2 layout). */
void orc_fill_ghosts(void *h, double t_s, double *padded_out) {
  orc_ctx *c = h;
  fill_ghosts(c, c->U, t_s / u_time());
  memcpy(padded_out, c->U, pad_cells(c) * NV * sizeof(double));
}

/* Inner-boundary primitive (SI) at time t_s for every (j, k): [8][nt][np]. */
void orc_inner_boundary(void *h, double t_s, double *out) {
  orc_ctx *c = h;
  double scale[NV] = {u_rho(), V_UNIT, V_UNIT, V_UNIT, u_pres(),
                      u_bfield(), u_bfield(), u_bfield()};
  size_t plane = (size_t)c->nt * c->np;
  for (int j = 0; j < c->nt; ++j)
    for (int k = 0; k < c->np; ++k) {
      double w[NV];
      inner_boundary_prim(c, t_s / u_time(), j, k, w);
      for (int v = 0; v < NV; ++v)
        out[v * plane + (size_t)j * c->np + k] = w[v] * scale[v];
    }
}

/* Clock: t [s], step, last dt [s], last residual, t [code units]. */
void orc_get_clock(const void *h, double *out) {
  const orc_ctx *c = h;
  out[0] = c->t * u_time();
  out[1] = (double)c->step;
  out[2] = c->last_dt * u_time();
  out[3] = c->last_resid;
  out[4] = c->t;
}

/* Restore a clock saved in code units (exact restart). */
void orc_set_clock_code(void *h, double t_code, long step) {
  orc_ctx *c = h;
  c->t = t_code;
  c->step = step;
}

void orc_set_clock(void *h, double t_s, long step) {
  orc_ctx *c = h;
  c->t = t_s / u_time();
  c->step = step;
}

/* Boundary-face integral of the last step, (dt/2) sum over both stages of
 * the outward area-weighted flux through non-periodic domain faces. */
void orc_last_boundary_flux(const void *h, double *out) {
  const orc_ctx *c = h;
  for (int v = 0; v < NV; ++v) out[v] = c->bflux[v];
}

/* Cell volumes (code units) of the active cells, [np][nt][nr]. */
void orc_volumes(const void *h, double *out) {
  const orc_ctx *c = h;
  double dph = c->pe[1] - c->pe[0], dth = c->te[1] - c->te[0];
  for (int k = 0; k < c->np; ++k)
    for (int j = 0; j < c->nt; ++j)
      for (int i = 0; i < c->nr; ++i) {
        size_t q = ((size_t)k * c->nt + j) * c->nr + i;
        double rm = c->re[i], rp = c->re[i + 1];
        if (c->geom == GEOM_SPH)
          out[q] = (rp * rp * rp - rm * rm * rm) / 3.0 *
                   (cos(c->te[j]) - cos(c->te[j + 1])) * dph;
        else
          out[q] = (rp - rm) * dth * dph;
      }
}

/* ---- initial state: radial expansion of the first map (Sect. 2.1) -------- */
/* rho ~ r^-2, v_r constant, v_t = 0, v_p' = -Omega r sin(theta) (plasma not
 * rotating in the inertial frame), p ~ r^(-2 gamma), B_r ~ r^-2, B_t = 0,
 * B_p ~ r^-1, scaled from the inner-boundary radius r_b = r_in. */
int orc_init_radial(void *h) {
  orc_ctx *c = h;
  if (c->n_maps < 1 || c->geom != GEOM_SPH) return -1;
  size_t plane = (size_t)c->nt * c->np;
  double rb = c->re[0];
  for (int k = 0; k < c->np; ++k)
    for (int j = 0; j < c->nt; ++j) {
      size_t q = (size_t)j * c->np + k;
      double wb[NV];
      for (int v = 0; v < NV; ++v) wb[v] = c->maps[(size_t)v * plane + q];
      for (int i = 0; i < c->nr; ++i) {
        double x = rb / c->rc[i], w[NV], u[NV];
        w[0] = wb[0] * x * x;
        w[1] = wb[1];
        w[2] = 0.0;
        w[3] = -c->omega * c->rc[i] * sin(c->tc[j]);
        w[4] = wb[4] * pow(x, 2.0 * c->gamma);
        w[5] = wb[5] * x * x;
        w[6] = 0.0;
        w[7] = wb[7] * x;
        prim_to_cons(c->gamma, w, u);
        for (int v = 0; v < NV; ++v) c->U[IX(c, v, i, j, k)] = u[v];
      }
    }
  if (c->tracer) memset(c->T, 0, pad_cells(c) * sizeof(double));
  return 0;
}

/* ---- passive CME tracer ---------------------------------------------------- */
/* tau [np][nt][nr] (dimensionless, 0 outside CME material) <-> rho tau */
int orc_set_tracer(void *h, const double *tau) {
  orc_ctx *c = h;
  if (!c->tracer) return -1;
  for (int k = 0; k < c->np; ++k)
    for (int j = 0; j < c->nt; ++j)
      for (int i = 0; i < c->nr; ++i)
        c->T[IX(c, 0, i, j, k)] = c->U[IX(c, 0, i, j, k)] *
                                  tau[((size_t)k * c->nt + j) * c->nr + i];
  return 0;
}

int orc_get_tracer(void *h, double *tau) {
  orc_ctx *c = h;
  if (!c->tracer) return -1;
  for (int k = 0; k < c->np; ++k)
    for (int j = 0; j < c->nt; ++j)
      for (int i = 0; i < c->nr; ++i)
        tau[((size_t)k * c->nt + j) * c->nr + i] =
            c->T[IX(c, 0, i, j, k)] / c->U[IX(c, 0, i, j, k)];
  return 0;
}

/* Boundary-face integral of the tracer flux (rho tau v . n dA, code units)
 * over the last step: the tracer content changes by minus this amount. */
double orc_tracer_flux(const void *h) { return ((const orc_ctx *)h)->tbflux; }

/* ---- velocity divergence diagnostic (Fig. 7) ------------------------------ */
/* Cell-centred finite-volume divergence of v (co-rotating frame) with face
 * velocities the mean of the two neighbouring cell centres; ghosts filled at
 * the current time (inner boundary map, zero-gradient outer boundary,
 * reflecting colatitude edges, periodic phi).  out [np][nt][nr] in 1/s. */
void orc_divv(void *h, double *out) {
  orc_ctx *c = h;
  fill_ghosts(c, c->U, c->t);
  double dth = c->te[1] - c->te[0], dph = c->pe[1] - c->pe[0];
  int di[3] = {1, 0, 0}, dj[3] = {0, 1, 0}, dk[3] = {0, 0, 1};
  for (int k = 0; k < c->np; ++k)
    for (int j = 0; j < c->nt; ++j)
      for (int i = 0; i < c->nr; ++i) {
        double vm[3], vp[3];
        for (int d = 0; d < 3; ++d) {
          double u0[NV], um[NV], up[NV], w0[NV], wm[NV], wp[NV];
          for (int v = 0; v < NV; ++v) {
            u0[v] = c->U[IX(c, v, i, j, k)];
            um[v] = c->U[IX(c, v, i - di[d], j - dj[d], k - dk[d])];
            up[v] = c->U[IX(c, v, i + di[d], j + dj[d], k + dk[d])];
          }
          cons_to_prim(c->gamma, u0, w0);
          cons_to_prim(c->gamma, um, wm);
          cons_to_prim(c->gamma, up, wp);
          vm[d] = 0.5 * (wm[1 + d] + w0[1 + d]);
          vp[d] = 0.5 * (w0[1 + d] + wp[1 + d]);
        }
        double rm = c->re[i], rp = c->re[i + 1];
        double div = (rp * rp * vp[0] - rm * rm * vm[0]) / c->volr[i] +
                     c->hr[i] * (c->se[j + 1] * vp[1] - c->se[j] * vm[1]) / c->ct[j] +
                     c->hr[i] * dth / (c->ct[j] * dph) * (vp[2] - vm[2]);
        out[((size_t)k * c->nt + j) * c->nr + i] = div / u_time();
      }
}

/* ---- probes (Sect. 2: sampling at moving locations, stretched grid) ------ */
/* traj: [n][npts][4] rows (t[s], r[m], theta[rad], phi_inertial[rad]) with
 * ascending t and unwrapped phi.  The location at the current time is the
 * linear interpolation in t (clamped), the co-rotating longitude is
 * phi - Omega t, and the primitives are trilinear in (r, theta, phi)
 * between the 8 surrounding active-cell centres (periodic in phi).
 * out: [n][12]: t, r, theta, phi', rho, v_r, v_t, v_p (inertial), p, B_r,
 * B_t, B_p, SI.  Locations outside the range of cell centres give NaN for
 * the 8 plasma values. */
void orc_sample(void *h, int n, int npts, const double *traj, double *out) {
  orc_ctx *c = h;
  double ts = c->t * u_time();
  double scale[NV] = {u_rho(), V_UNIT, V_UNIT, V_UNIT, u_pres(),
                      u_bfield(), u_bfield(), u_bfield()};
  double twopi = 2.0 * 3.14159265358979323846;
  for (int q = 0; q < n; ++q) {
    const double *tb = traj + (size_t)q * npts * 4;
    double pos[4];
    if (npts == 1 || ts <= tb[0]) {
      memcpy(pos, tb, sizeof pos);
    } else if (ts >= tb[(npts - 1) * 4]) {
      memcpy(pos, tb + (npts - 1) * 4, sizeof pos);
    } else {
      int m = 0;
      while (m + 1 < npts - 1 && tb[(m + 1) * 4] <= ts) ++m;
      double a = (ts - tb[m * 4]) / (tb[(m + 1) * 4] - tb[m * 4]);
      for (int e = 1; e < 4; ++e)
        pos[e] = (1.0 - a) * tb[m * 4 + e] + a * tb[(m + 1) * 4 + e];
    }
    double r = pos[1] / u_len(), th = pos[2];
    double ph = pos[3] - c->omega * c->t;
    ph = ph - floor(ph / twopi) * twopi;
    double *o = out + (size_t)q * 12;
    o[0] = ts;
    o[1] = pos[1];
    o[2] = th;
    o[3] = ph;
    int nr = c->nr, nt = c->nt, np = c->np;
    if (!(r >= c->rc[0] && r <= c->rc[nr - 1] && th >= c->tc[0] &&
          th <= c->tc[nt - 1])) {
      for (int v = 0; v < NV; ++v) o[4 + v] = NAN;
      continue;
    }
    int i = 0;
    while (i + 1 < nr - 1 && c->rc[i + 1] <= r) ++i;
    int j = 0;
    while (j + 1 < nt - 1 && c->tc[j + 1] <= th) ++j;
    double dph = c->pe[1] - c->pe[0];
    double fk = (ph - c->pc[0]) / dph;
    int k0 = (int)floor(fk);
    double az = fk - k0;
    int ka = ((k0 % np) + np) % np, kb = (ka + 1) % np;
    double ax = (r - c->rc[i]) / (c->rc[i + 1] - c->rc[i]);
    double ay = (th - c->tc[j]) / (c->tc[j + 1] - c->tc[j]);
    double acc[NV] = {0};
    for (int cz = 0; cz < 2; ++cz)
      for (int cy = 0; cy < 2; ++cy)
        for (int cx = 0; cx < 2; ++cx) {
          double wt = (cx ? ax : 1.0 - ax) * (cy ? ay : 1.0 - ay) *
                      (cz ? az : 1.0 - az);
          double u[NV], w[NV];
          for (int v = 0; v < NV; ++v)
            u[v] = c->U[IX(c, v, i + cx, j + cy, cz ? kb : ka)];
          cons_to_prim(c->gamma, u, w);
          for (int v = 0; v < NV; ++v) acc[v] += wt * w[v];
        }
    acc[3] += c->omega * r * sin(th); /* to the inertial frame */
    for (int v = 0; v < NV; ++v) o[4 + v] = acc[v] * scale[v];
  }
}

/* ---- div B diagnostic ----------------------------------------------------- */
/* Cell-centred finite-volume divergence with face B the mean of the two
 * adjacent centres, normalised |div B| h / |B| with h = min(dx_d).
 * Ghosts must have been filled (call orc_fill_ghosts first). */
void orc_divb(void *h, double *out) {
  orc_ctx *c = h;
  double dth = c->te[1] - c->te[0], dph = c->pe[1] - c->pe[0];
  for (int k = 0; k < c->np; ++k)
    for (int j = 0; j < c->nt; ++j)
      for (int i = 0; i < c->nr; ++i) {
        size_t q = ((size_t)k * c->nt + j) * c->nr + i;
        double b[3], bm[3], bp[3];
        int di[3] = {1, 0, 0}, dj[3] = {0, 1, 0}, dk[3] = {0, 0, 1};
        double div = 0.0;
        double rm = c->re[i], rp = c->re[i + 1];
        double vr = (rp * rp * rp - rm * rm * rm) / 3.0;
        double hr = (rp * rp - rm * rm) / (2.0 * vr);
        double ct = cos(c->te[j]) - cos(c->te[j + 1]);
        for (int d = 0; d < 3; ++d) {
          b[d] = c->U[IX(c, 5 + d, i, j, k)];
          bm[d] = 0.5 * (b[d] + c->U[IX(c, 5 + d, i - di[d], j - dj[d],
                                        k - dk[d])]);
          bp[d] = 0.5 * (b[d] + c->U[IX(c, 5 + d, i + di[d], j + dj[d],
                                        k + dk[d])]);
        }
        double hmin;
        if (c->geom == GEOM_SPH) {
          div = (rp * rp * bp[0] - rm * rm * bm[0]) / vr +
                hr * (sin(c->te[j + 1]) * bp[1] - sin(c->te[j]) * bm[1]) / ct +
                hr * dth / (ct * dph) * (bp[2] - bm[2]);
          hmin = rp - rm;
          double h2 = c->rc[i] * dth, h3 = c->rc[i] * sin(c->tc[j]) * dph;
          if (h2 < hmin) hmin = h2;
          if (h3 < hmin) hmin = h3;
        } else {
          double hx = c->re[1] - c->re[0];
          div = (bp[0] - bm[0]) / hx + (bp[1] - bm[1]) / dth +
                (bp[2] - bm[2]) / dph;
          hmin = hx < dth ? hx : dth;
          if (dph < hmin) hmin = dph;
        }
        double bn = sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
        out[q] = bn > 0.0 ? fabs(div) * hmin / bn : 0.0;
      }
}

/* OpenMP threads the oracle's parallel loops use, and setting them (the
 * CPU-baseline timing reports the count actually used). */
int orc_threads(void) { return omp_get_max_threads(); }
void orc_set_threads(int n) {
  if (n > 0) omp_set_num_threads(n);
}

/* Right-hand side of one stage on a caller-set padded state (ghost layers
 * included, bc_mode frozen): L = -div F + S of every active cell, [8][np][nt][nr]
 * in code units (LT, the tracer's, [np][nt][nr], when the oracle carries the
 * tracer and T is given), and the fluxes through the six faces of the active
 * box (layout of compute_rhs_bf).  A block of a refined grid is stepped by
 * calling this on its padded state and combining the stages outside. */
int orc_rhs(void *h, const double *Upad, const double *Tpad, double *L_out,
            double *LT_out, double *bf) {
  orc_ctx *c = h;
  int nr = c->nr, nt = c->nt, np = c->np;
  size_t n = pad_cells(c);
  double bnd[NV], tb = 0.0;
  memcpy(c->U0, Upad, n * NV * sizeof(double));
  int trc = c->tracer && Tpad;
  if (trc) memcpy(c->T0, Tpad, n * sizeof(double));
  compute_rhs_bf(c, c->U0, c->L, bnd, trc ? c->T0 : 0, c->LT, &tb, c->t, bf);
  size_t act = (size_t)nr * nt * np;
  for (int k = 0; k < np; ++k)
    for (int j = 0; j < nt; ++j)
      for (int i = 0; i < nr; ++i) {
        size_t q = ((size_t)k * nt + j) * nr + i;
        for (int v = 0; v < NV; ++v) L_out[v * act + q] = c->L[IX(c, v, i, j, k)];
        if (trc && LT_out) LT_out[q] = c->LT[IX(c, 0, i, j, k)];
      }
  return 0;
}
