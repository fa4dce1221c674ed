/*
 * FP64 CPU ORACLE of the M1 Lyman-alpha transfer step.
 *
 * TEST INFRASTRUCTURE ONLY: this file exists to check the GPU library.  Only
 * tests, the smoke check and the CPU-baseline leg of the benchmark may build,
 * load or call it.  It shares no code with the GPU path.
 *
 * Plain, slow, obviously correct: scalar double loops written from the paper
 * (Nebrin et al., "Lyman-alpha pressure strongly enhances pre-supernova
 * feedback at cosmic dawn", Section 2.1 and Appendix A).  OpenMP only spreads
 * independent bins (advection) or independent cells (frequency step) over
 * threads; it never changes the arithmetic of a cell.
 *
 * State variables (per cell and frequency bin k): E_k = 4 pi J_k / c and
 * F_k = 4 pi H_k / c, i.e. spectral energy density and flux over c.
 * Layout of every per-bin array: [k][j][i], cell index c = j*nx + i.
 *
 * One call of oracle_step() advances n -> n+1:
 *   (0) optional active-bin selection (Section 2.2, active bins): with
 *       active_frac > 0 only bins holding more than that fraction of the
 *       total Lyman-alpha energy in the volume are advected in (1);
 *   (1) advection step per bin (Section 2.1, step 1): MinMod-limited linear
 *       reconstruction of E and f = F/E, Levermore closure, GLF flux blended
 *       with the diffusion flux by epsilon(tau), upwind velocity advection,
 *       radiation-pressure work term, explicit Euler update, causality clamp;
 *   (2) implicit emission/absorption step (Section 2.1, step 2, BDF1), in
 *       one substep, or with substep_rule set, per cell in substeps accepted
 *       when the cell's energy density changes by less than 10 % (halved and
 *       redone otherwise);
 *   (3) radiation force density (Section 2.3), f = sum_k dnu_k alpha_F,k F_k
 *       (with substeps: the substep forces sum_k dnu_k (F. - F..)/(c dt_sub)
 *       averaged over the step);
 *   (4) implicit frequency step per cell (Section 2.1, step 3; Appendix A):
 *       exponential-scheme leakage coefficients, tridiagonal solve
 *       (Thomas algorithm in long double), H rescaled by J_new/J_old.
 *
 * With `band` set the same step moves broad bands instead (Section 2.5,
 * Appendix E): (1) unchanged with the band's flux opacity in the blend,
 * (2) with the band's absorption opacity and emission, (3) the force
 * sum_B kappa_F,B F_B, and no step (4).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define C_LIGHT 2.99792458e10
#define ORACLE_PI 3.14159265358979323846

typedef struct {
  int nx, ny, nb;
  int geom;          /* 0: 2D Cartesian slab (unit depth), 1: cylindrical (R,z) */
  int bc[4];         /* x-, x+, y-, y+ : 0 vacuum, 1 reflecting */
  int recoil, doppler;
  double c_tilde, dt;
  const double *xe, *ye;     /* cell edges [nx+1], [ny+1] */
  const double *nu_c, *dnu;  /* bin centres (absolute, Hz) and widths [nb] */
  const double *alpha;       /* line-centre opacity n_HI sigma0(T) [ncell] */
  const double *acabs;       /* continuum absorption alpha_c (1-omega) */
  const double *acF;         /* continuum flux opacity alpha_c (1-omega g) */
  const double *pd;          /* destruction probability */
  const double *ux, *uy;     /* gas velocity */
  const double *dnuD;        /* Doppler width of the cell [Hz] */
  const double *hkT;         /* h / (k_B T) [s] */
  const double *emis;        /* Lya luminosity density [erg/s/cm^3] */
  const int *cls;            /* temperature class of the cell [ncell] */
  const double *hbar;        /* bin-averaged Voigt <H>_k per class [ncls][nb] */
  const double *phi;         /* bin-averaged emission profile per class [ncls][nb] */
  double active_frac;        /* 0: advect every bin; > 0: only bins whose energy
                                exceeds this fraction of the total (Section 2.2,
                                active bins) */
  int *active;               /* [nb] out: 1 where bin k was advected this step */
  int substep_rule;          /* 1: emission/absorption in substeps under the
                                10 % energy rule (Section 2.1, step 2) */
  int *substeps;             /* [ncell] out (may be NULL): accepted substeps of
                                each cell in the last step */
  double *sub_margin;        /* [ncell] out (may be NULL): over the attempts of
                                the last step, the smallest |r/0.1 - 1|, r the
                                attempt's relative energy change (how close a
                                decision came to the 10 % boundary) */
  /* Broad-band transport (Section 2.5 and Appendix E: stellar and IR bands): with band set,
   * each of the nb "bins" is a band B with per-cell absorption opacity
   * kappa_abs, flux opacity kappa_F [cm^-1] and luminosity density
   * [erg/s/cm^3], tables [nb][ncell]; the line data above (alpha, hbar,
   * phi, cls, pd, acabs, acF, emis, nu_c, dnu, dnuD, hkT) are not used, and
   * there is no frequency step (no frequency-derivative terms). */
  int band;
  const double *kabs, *kflux, *jband;
  /* Interface flux: 0 the corrected GLF flux the paper adopts (HLL with
   * signal speeds -c_tilde, +c_tilde); 1 the HLL flux with the extreme
   * eigenvalues of the M1 system as signal speeds, which the paper reports
   * having tried (Section 2.1, footnote on the GLF solver), with the same
   * eps blend: eps times its dissipation in the F flux, eps times the whole
   * flux plus (1 - eps) times the diffusion flux for E. */
  int flux;
} OracleProblem;

/* ------------------------------------------------------------------------ */
/* Levermore closure (Section 2.1): chi(f) = (3 + 4 f^2)/(5 + 2 sqrt(4 - 3 f^2)),
 * D = (1-chi)/2 I + (3 chi - 1)/2 h (x) h, h = F/|F|.  Dpp is the azimuthal
 * (cylindrical) or out-of-plane (slab) diagonal entry, (1-chi)/2. */
static double levermore_chi(double f) {
  return (3.0 + 4.0 * f * f) / (5.0 + 2.0 * sqrt(4.0 - 3.0 * f * f));
}

static void eddington_tensor(double E, double Fx, double Fy,
                             double *Dxx, double *Dyy, double *Dxy, double *Dpp) {
  double nF = hypot(Fx, Fy);      /* |F| without underflow of the squares */
  double f = (E > 0.0) ? nF / E : 0.0;
  if (f > 1.0) f = 1.0;
  double chi = levermore_chi(f);
  double iso = 0.5 * (1.0 - chi), dir = 0.5 * (3.0 * chi - 1.0);
  double hx = 0.0, hy = 0.0;
  if (nF > 0.0) { hx = Fx / nF; hy = Fy / nF; }
  *Dxx = iso + dir * hx * hx;
  *Dyy = iso + dir * hy * hy;
  *Dxy = dir * hx * hy;
  *Dpp = iso;
}

/* Signal speeds of the M1 system across a face with normal n (0: x, 1: y),
 * in units of the transport speed: the smallest and largest eigenvalues of
 * the Jacobian of the face flux (F_n, P_nx, P_ny) with respect to
 * (E, F_x, F_y), where P = D(f) E with the Levermore closure of reduced flux
 * f = (fx, fy), |f| <= 1.  Write D = a(q) I + w(q) f (x) f with q = f^2,
 * a = (1 - chi)/2 and w = (3 chi - 1)/(2 q) = 3 / (2 + sqrt(4 - 3 q)) (the
 * second form follows from chi and stays finite at q = 0).  P is homogeneous
 * of degree one in (E, F), so dP_nm/dE = D_nm - f . grad_f D_nm and
 * dP_nm/dF_k = dD_nm/df_k.  The eigenvalues are the roots of the
 * characteristic cubic (trace, principal minors, determinant), all real for
 * this hyperbolic system, found in long double by the trigonometric method.
 * Where |f| -> 1 the three roots merge at f . n and the cubic's roots lose
 * accuracy like the cube root of the rounding. */
static void signal_speeds(double fx_d, double fy_d, int n, double *lmin, double *lmax) {
  long double f[2] = {fx_d, fy_d};
  long double q = f[0] * f[0] + f[1] * f[1];
  if (q > 1.0L) q = 1.0L;
  long double s = sqrtl(4.0L - 3.0L * q);
  long double chi = (3.0L + 4.0L * q) / (5.0L + 2.0L * s);
  long double dchi = (4.0L * (5.0L + 2.0L * s) + 3.0L * (3.0L + 4.0L * q) / s) /
                     ((5.0L + 2.0L * s) * (5.0L + 2.0L * s));       /* d chi / d q */
  long double a = 0.5L * (1.0L - chi), da = -0.5L * dchi;
  long double w = 3.0L / (2.0L + s), dw = 9.0L / (2.0L * s * (2.0L + s) * (2.0L + s));
  long double J[3][3];
  J[0][0] = 0.0L; J[0][1] = (n == 0); J[0][2] = (n == 1);
  for (int m = 0; m < 2; ++m) {
    long double Dnm = (n == m ? a : 0.0L) + w * f[n] * f[m];
    long double dD[2];
    for (int k = 0; k < 2; ++k)
      dD[k] = 2.0L * f[k] * ((n == m ? da : 0.0L) + dw * f[n] * f[m]) +
              w * ((n == k ? f[m] : 0.0L) + (m == k ? f[n] : 0.0L));
    J[1 + m][0] = Dnm - f[0] * dD[0] - f[1] * dD[1];
    J[1 + m][1] = dD[0];
    J[1 + m][2] = dD[1];
  }
  /* lambda^3 + A lambda^2 + B lambda + C = 0 */
  long double tr = J[0][0] + J[1][1] + J[2][2];
  long double mi = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) +
                   (J[0][0] * J[2][2] - J[0][2] * J[2][0]) +
                   (J[1][1] * J[2][2] - J[1][2] * J[2][1]);
  long double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                    J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                    J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  long double A = -tr, B = mi, C = -det;
  long double p = B - A * A / 3.0L;
  long double r = 2.0L * A * A * A / 27.0L - A * B / 3.0L + C;
  long double shift = -A / 3.0L;
  if (p >= 0.0L) {                   /* a triple root (p = 0 up to rounding) */
    *lmin = *lmax = (double)shift;
    return;
  }
  long double m2 = 2.0L * sqrtl(-p / 3.0L);
  long double arg = 3.0L * r / (p * m2);        /* cos(3 theta) */
  if (arg > 1.0L) arg = 1.0L;
  if (arg < -1.0L) arg = -1.0L;
  long double th = acosl(arg) / 3.0L;
  const long double two_pi_3 = 2.0943951023931954923084289221863353L;
  *lmax = (double)(shift + m2 * cosl(th));
  *lmin = (double)(shift + m2 * cosl(th - 2.0L * two_pi_3));
}

/* MinMod of two slopes (sign comparison, so products never underflow). */
static double minmod(double a, double b) {
  if (a > 0.0 && b > 0.0) return a < b ? a : b;
  if (a < 0.0 && b < 0.0) return a > b ? a : b;
  return 0.0;
}

/* ------------------------------------------------------------------------ */
/* Geometry.  Cylindrical cell centroid along R: volume centroid
 * (2/3)(R+^3 - R-^3)/(R+^2 - R-^2); along z and in the slab: midpoint. */
typedef struct {
  int nx, ny;
  double *xcp, *ycp;   /* centroids incl. 2 ghost layers: [nx+4], [ny+4] */
} Geometry;

static double centroid_R(double a, double b) {
  return (2.0 / 3.0) * (b * b * b - a * a * a) / (b * b - a * a);
}

static void build_geometry(const OracleProblem *P, Geometry *G) {
  int nx = P->nx, ny = P->ny;
  G->nx = nx; G->ny = ny;
  G->xcp = (double *)malloc(sizeof(double) * (nx + 4));
  G->ycp = (double *)malloc(sizeof(double) * (ny + 4));
  double dx = P->xe[1] - P->xe[0], dxr = P->xe[nx] - P->xe[nx - 1];
  for (int i = 0; i < nx; ++i)
    G->xcp[i + 2] = (P->geom == 1) ? centroid_R(P->xe[i], P->xe[i + 1])
                                   : 0.5 * (P->xe[i] + P->xe[i + 1]);
  for (int j = 0; j < ny; ++j) G->ycp[j + 2] = 0.5 * (P->ye[j] + P->ye[j + 1]);
  /* ghosts: reflecting = mirror image of the interior centroid;
   * vacuum = centroid of the cell continued past the edge. */
  for (int g = 1; g <= 2; ++g) {
    /* x- */
    if (P->bc[0] == 1) G->xcp[2 - g] = 2.0 * P->xe[0] - G->xcp[2 + g - 1];
    else {
      double a = P->xe[0] - g * dx, b = a + dx;
      G->xcp[2 - g] = (P->geom == 1) ? centroid_R(a, b) : 0.5 * (a + b);
    }
    /* x+ */
    if (P->bc[1] == 1) G->xcp[nx + 1 + g] = 2.0 * P->xe[nx] - G->xcp[nx + 2 - g];
    else {
      double a = P->xe[nx] + (g - 1) * dxr, b = a + dxr;
      G->xcp[nx + 1 + g] = (P->geom == 1) ? centroid_R(a, b) : 0.5 * (a + b);
    }
  }
  double dy = P->ye[1] - P->ye[0], dyt = P->ye[ny] - P->ye[ny - 1];
  for (int g = 1; g <= 2; ++g) {
    if (P->bc[2] == 1) G->ycp[2 - g] = 2.0 * P->ye[0] - G->ycp[2 + g - 1];
    else G->ycp[2 - g] = P->ye[0] - (g - 0.5) * dy;
    if (P->bc[3] == 1) G->ycp[ny + 1 + g] = 2.0 * P->ye[ny] - G->ycp[ny + 2 - g];
    else G->ycp[ny + 1 + g] = P->ye[ny] + (g - 0.5) * dyt;
  }
}

static void free_geometry(Geometry *G) { free(G->xcp); free(G->ycp); }

/* Face areas and cell volume (cylindrical: 2 pi R dz, pi (R+^2 - R-^2), and
 * pi (R+^2 - R-^2) dz; slab: unit depth). */
static double area_x(const OracleProblem *P, int iface, int j) {
  double dz = P->ye[j + 1] - P->ye[j];
  return (P->geom == 1) ? 2.0 * ORACLE_PI * P->xe[iface] * dz : dz;
}
static double area_y(const OracleProblem *P, int i) {
  double a = P->xe[i], b = P->xe[i + 1];
  return (P->geom == 1) ? ORACLE_PI * (b * b - a * a) : (b - a);
}
static double cell_volume(const OracleProblem *P, int i, int j) {
  return area_y(P, i) * (P->ye[j + 1] - P->ye[j]);
}

/* ------------------------------------------------------------------------ */
/* Padded copies of one bin (2 ghost layers) with the boundary rules:
 * vacuum  : E = F = 0, alpha_F = 0, velocity copied from the boundary cell;
 * reflect : mirror image, normal components of f and u negated.            */
typedef struct {
  int px;                 /* padded row length nx+4 */
  double *E, *fx, *fy, *aF;
} PadBin;

static int mirror(int i, int n) { return (i < 0) ? (-1 - i) : (2 * n - 1 - i); }

static void fill_padded_bin(const OracleProblem *P, int k, const double *E,
                            const double *Fx, const double *Fy, PadBin *B) {
  int nx = P->nx, ny = P->ny, px = nx + 4;
  size_t nc = (size_t)nx * ny;
  const double *Ek = E + (size_t)k * nc, *Xk = Fx + (size_t)k * nc, *Yk = Fy + (size_t)k * nc;
  for (int jp = 0; jp < ny + 4; ++jp)
    for (int ip = 0; ip < px; ++ip) {
      int i = ip - 2, j = jp - 2;
      size_t q = (size_t)jp * px + ip;
      B->E[q] = B->fx[q] = B->fy[q] = B->aF[q] = 0.0;
      int gx = (i < 0 || i >= nx), gy = (j < 0 || j >= ny);
      if (gx && gy) continue;                       /* corners never used */
      int si = i, sj = j;
      double sgx = 1.0, sgy = 1.0;
      if (gx) {
        int side = (i < 0) ? 0 : 1;
        if (P->bc[side] != 1) continue;             /* vacuum */
        si = mirror(i, nx); sgx = -1.0;
      }
      if (gy) {
        int side = (j < 0) ? 2 : 3;
        if (P->bc[side] != 1) continue;
        sj = mirror(j, ny); sgy = -1.0;
      }
      size_t c = (size_t)sj * nx + si;
      double e = Ek[c];
      B->E[q] = e;
      B->fx[q] = (e > 0.0) ? sgx * Xk[c] / e : 0.0;
      B->fy[q] = (e > 0.0) ? sgy * Yk[c] / e : 0.0;
      B->aF[q] = P->band ? P->kflux[(size_t)k * nc + c]
                         : P->alpha[c] * P->hbar[(size_t)P->cls[c] * P->nb + k] + P->acF[c];
    }
}

/* Face-normal velocity: mean of the two adjacent cell velocities (ghosts:
 * copy at vacuum, mirror at reflecting boundaries).  dir 0: x-face with
 * iface in [0, nx]; dir 1: y-face with jface in [0, ny]. */
static void face_velocity(const OracleProblem *P, int dir, int a, int b,
                          double *un, double *ut) {
  int nx = P->nx, ny = P->ny;
  if (dir == 0) {            /* x-face a = iface, b = j */
    int il = a - 1, ir = a, j = b;
    double uxl, uyl, uxr, uyr;
    if (il < 0) {
      size_t c = (size_t)j * nx;
      uxl = (P->bc[0] == 1) ? -P->ux[c] : P->ux[c]; uyl = P->uy[c];
    } else { size_t c = (size_t)j * nx + il; uxl = P->ux[c]; uyl = P->uy[c]; }
    if (ir >= nx) {
      size_t c = (size_t)j * nx + nx - 1;
      uxr = (P->bc[1] == 1) ? -P->ux[c] : P->ux[c]; uyr = P->uy[c];
    } else { size_t c = (size_t)j * nx + ir; uxr = P->ux[c]; uyr = P->uy[c]; }
    *un = 0.5 * (uxl + uxr); *ut = 0.5 * (uyl + uyr);
  } else {                   /* y-face a = jface, b = i */
    int jl = a - 1, jr = a, i = b;
    double uxl, uyl, uxr, uyr;
    if (jl < 0) {
      size_t c = (size_t)i;
      uyl = (P->bc[2] == 1) ? -P->uy[c] : P->uy[c]; uxl = P->ux[c];
    } else { size_t c = (size_t)jl * nx + i; uxl = P->ux[c]; uyl = P->uy[c]; }
    if (jr >= ny) {
      size_t c = (size_t)(ny - 1) * nx + i;
      uyr = (P->bc[3] == 1) ? -P->uy[c] : P->uy[c]; uxr = P->ux[c];
    } else { size_t c = (size_t)jr * nx + i; uxr = P->ux[c]; uyr = P->uy[c]; }
    *un = 0.5 * (uyl + uyr); *ut = 0.5 * (uxl + uxr);
  }
}

/* Velocity-gradient pieces of cell (i,j) (Appendix A): d(u_x)/dx, d(u_y)/dx,
 * d(u_x)/dy, d(u_y)/dy from face velocities, and <u_R/R> (cylindrical). */
typedef struct { double dxux, dxuy, dyux, dyuy, uR_R; } VelGrad;

static VelGrad velocity_gradient(const OracleProblem *P, int i, int j) {
  VelGrad g;
  double unp, utp, unm, utm;
  face_velocity(P, 0, i + 1, j, &unp, &utp);
  face_velocity(P, 0, i, j, &unm, &utm);
  double hx = P->xe[i + 1] - P->xe[i];
  g.dxux = (unp - unm) / hx;
  g.dxuy = (utp - utm) / hx;
  g.uR_R = (P->geom == 1) ? (unp + unm) / (P->xe[i + 1] + P->xe[i]) : 0.0;
  face_velocity(P, 1, j + 1, i, &unp, &utp);
  face_velocity(P, 1, j, i, &unm, &utm);
  double hy = P->ye[j + 1] - P->ye[j];
  g.dyuy = (unp - unm) / hy;
  g.dyux = (utp - utm) / hy;
  return g;
}

/* D : grad u (Appendix A; slab analogue without the azimuthal term). */
static double D_colon_gradu(const OracleProblem *P, double E, double Fx, double Fy,
                            const VelGrad *g) {
  double Dxx, Dyy, Dxy, Dpp;
  eddington_tensor(E, Fx, Fy, &Dxx, &Dyy, &Dxy, &Dpp);
  double s = Dxx * g->dxux + Dyy * g->dyuy + Dxy * (g->dyux + g->dxuy);
  if (P->geom == 1) s += Dpp * g->uR_R;
  return s;
}

/* ------------------------------------------------------------------------ */
/* Interface flux of one bin through one face.
 * Inputs are the padded-array indices of the left (lower coordinate) and
 * right cells plus the two outer neighbours used by the MinMod slopes.
 * n selects the normal direction (0: x, 1: y).  Returns the fluxes of E, F_x
 * and F_y (per unit area, in units where the transport speed is 1, i.e. the
 * caller multiplies by c_tilde dt A / dV). */
typedef struct { double e, fx, fy; } Flux3;

static Flux3 face_flux(const PadBin *B, const double *xcent, double xf,
                       size_t qLL, size_t qL, size_t qR, size_t qRR,
                       int iL, int iR, int n, double u_n, int flux) {
  /* centroid coordinates along the normal: xcent indexed by padded index */
  double xLL = xcent[iL - 1], xL = xcent[iL], xR = xcent[iR], xRR = xcent[iR + 1];
  const double *q[3] = {B->E, B->fx, B->fy};
  double sL[3], sR[3];
  for (int v = 0; v < 3; ++v) {
    double aLL = q[v][qLL], aL = q[v][qL], aR = q[v][qR], aRR = q[v][qRR];
    sL[v] = minmod((aL - aLL) / (xL - xLL), (aR - aL) / (xR - xL));
    sR[v] = minmod((aR - aL) / (xR - xL), (aRR - aR) / (xRR - xR));
  }
  /* reconstructed face states */
  double EL = B->E[qL] + sL[0] * (xf - xL);
  double fxL = B->fx[qL] + sL[1] * (xf - xL);
  double fyL = B->fy[qL] + sL[2] * (xf - xL);
  double ER = B->E[qR] + sR[0] * (xf - xR);
  double fxR = B->fx[qR] + sR[1] * (xf - xR);
  double fyR = B->fy[qR] + sR[2] * (xf - xR);
  /* |f| > 1 at the interface: scale the components down to unit length */
  double nL = sqrt(fxL * fxL + fyL * fyL), nR = sqrt(fxR * fxR + fyR * fyR);
  if (nL > 1.0) { fxL /= nL; fyL /= nL; }
  if (nR > 1.0) { fxR /= nR; fyR /= nR; }
  double FxL = fxL * EL, FyL = fyL * EL, FxR = fxR * ER, FyR = fyR * ER;
  /* Eddington tensors of the face states: P = D(f) E */
  double Dxx, Dyy, Dxy, Dpp;
  eddington_tensor(1.0, fxL, fyL, &Dxx, &Dyy, &Dxy, &Dpp);
  double PnxL = (n == 0 ? Dxx : Dxy) * EL, PnyL = (n == 0 ? Dxy : Dyy) * EL;
  eddington_tensor(1.0, fxR, fyR, &Dxx, &Dyy, &Dxy, &Dpp);
  double PnxR = (n == 0 ? Dxx : Dxy) * ER, PnyR = (n == 0 ? Dxy : Dyy) * ER;
  /* flux optical depth between the centroids and the blending factor */
  double tau = B->aF[qL] * (xf - xL) + B->aF[qR] * (xR - xf);
  double eps = (0.2 + tau) / (0.2 + tau + tau * tau);
  /* (1 - eps)/(3 tau), rewritten as tau / (3 (0.2 + tau + tau^2)) so that it
   * is finite at tau = 0 */
  double dcoef = tau / (3.0 * (0.2 + tau + tau * tau));
  double FnL = (n == 0) ? FxL : FyL, FnR = (n == 0) ? FxR : FyR;
  Flux3 r;
  if (flux == 1) {
    /* HLL with the M1 signal speeds: the central part
     * (sR G_L - sL G_R)/(sR - sL) and the dissipation sL sR (U_R - U_L)/(sR - sL),
     * sL = min(0, lambda_min of both states), sR = max(0, lambda_max of both) */
    double lminL, lmaxL, lminR, lmaxR;
    signal_speeds(fxL, fyL, n, &lminL, &lmaxL);
    signal_speeds(fxR, fyR, n, &lminR, &lmaxR);
    double sL = lminL < lminR ? lminL : lminR, sR = lmaxL > lmaxR ? lmaxL : lmaxR;
    if (sL > 0.0) sL = 0.0;
    if (sR < 0.0) sR = 0.0;
    double GL[3] = {FnL, PnxL, PnyL}, GR[3] = {FnR, PnxR, PnyR};
    double UL[3] = {EL, FxL, FyL}, UR[3] = {ER, FxR, FyR};
    double cen[3], dis[3];
    for (int v = 0; v < 3; ++v) {
      if (sR - sL > 0.0) {
        cen[v] = (sR * GL[v] - sL * GR[v]) / (sR - sL);
        dis[v] = sL * sR * (UR[v] - UL[v]) / (sR - sL);
      } else {                     /* both speeds zero: no wave crosses the face */
        cen[v] = 0.5 * (GL[v] + GR[v]);
        dis[v] = 0.0;
      }
    }
    r.e = eps * (cen[0] + dis[0]) - dcoef * (B->E[qR] - B->E[qL]);
    r.fx = cen[1] + eps * dis[1];
    r.fy = cen[2] + eps * dis[2];
  } else {
    r.e = eps * (0.5 * (FnL + FnR) - 0.5 * (ER - EL)) - dcoef * (B->E[qR] - B->E[qL]);
    r.fx = 0.5 * (PnxL + PnxR) - eps * 0.5 * (FxR - FxL);
    r.fy = 0.5 * (PnyL + PnyR) - eps * 0.5 * (FyR - FyL);
  }
  /* upwind velocity advection with the reconstructed upstream state */
  double b = u_n / C_LIGHT;
  if (u_n > 0.0) { r.e += b * EL; r.fx += b * FxL; r.fy += b * FyL; }
  else if (u_n < 0.0) { r.e += b * ER; r.fx += b * FxR; r.fy += b * FyR; }
  return r;
}

/* Advection + emission/absorption of bin k; writes E**, F** of the bin. */
/* Static velocity data of a step: face-normal velocities and cell gradients. */
typedef struct {
  double *unx;      /* x-face normal velocity [ny][nx+1] */
  double *uny;      /* y-face normal velocity [ny+1][nx] */
  VelGrad *grad;    /* [ncell] */
} VelData;

static void build_velocity(const OracleProblem *P, VelData *V) {
  int nx = P->nx, ny = P->ny;
  V->unx = (double *)malloc(sizeof(double) * (size_t)(nx + 1) * ny);
  V->uny = (double *)malloc(sizeof(double) * (size_t)nx * (ny + 1));
  V->grad = (VelGrad *)malloc(sizeof(VelGrad) * (size_t)nx * ny);
  double ut;
  for (int j = 0; j < ny; ++j)
    for (int f = 0; f <= nx; ++f) face_velocity(P, 0, f, j, &V->unx[(size_t)j * (nx + 1) + f], &ut);
  for (int f = 0; f <= ny; ++f)
    for (int i = 0; i < nx; ++i) face_velocity(P, 1, f, i, &V->uny[(size_t)f * nx + i], &ut);
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) V->grad[(size_t)j * nx + i] = velocity_gradient(P, i, j);
}

static void free_velocity(VelData *V) { free(V->unx); free(V->uny); free(V->grad); }

/* Opacities and source of cell c in bin (or band) k for step (2): kE the
 * absorption coefficient of E, aF that of F, src the emission term j/c. */
static void source_coeffs(const OracleProblem *P, int k, size_t c, double *kE, double *aF,
                          double *src) {
  size_t nc = (size_t)P->nx * P->ny, ck = (size_t)k * nc + c;
  if (P->band) {
    *kE = P->kabs[ck];
    *aF = P->kflux[ck];
    *src = P->jband[ck] / C_LIGHT;
    return;
  }
  double h = P->hbar[(size_t)P->cls[c] * P->nb + k];
  double aH = P->alpha[c] * h;
  *kE = P->acabs[c] + P->pd[c] * aH;
  *aF = aH + P->acF[c];
  *src = P->emis[c] * P->phi[(size_t)P->cls[c] * P->nb + k] / C_LIGHT;
}

/* Advection (when `advect`) and emission/absorption of bin k.  A bin that is
 * not advected keeps its state through step (1): no fluxes, no work or hoop
 * term, no clamp (the state is causal already); step (2) acts as usual. */
static void advect_source_bin(const OracleProblem *P, const Geometry *G,
                              const VelData *V, int k, int advect, int source,
                              const double *E, const double *Fx, const double *Fy,
                              double *Eo, double *Fxo, double *Fyo, PadBin *B,
                              Flux3 *fxf, Flux3 *fyf) {
  int nx = P->nx, ny = P->ny, px = nx + 4;
  size_t nc = (size_t)nx * ny;
  double ctdt = P->c_tilde * P->dt;
  if (!advect) {
    for (size_t c = 0; c < nc; ++c) {
      size_t ck = (size_t)k * nc + c;
      if (!source) { Eo[ck] = E[ck]; Fxo[ck] = Fx[ck]; Fyo[ck] = Fy[ck]; continue; }
      double kE, aF, src;
      source_coeffs(P, k, c, &kE, &aF, &src);
      Eo[ck] = (E[ck] + ctdt * src) / (1.0 + ctdt * kE);
      Fxo[ck] = Fx[ck] / (1.0 + ctdt * aF);
      Fyo[ck] = Fy[ck] / (1.0 + ctdt * aF);
    }
    return;
  }
  fill_padded_bin(P, k, E, Fx, Fy, B);
  /* x-faces: iface = 0..nx between cells iface-1 and iface */
  for (int j = 0; j < ny; ++j)
    for (int f = 0; f <= nx; ++f) {
      int iL = f - 1 + 2, iR = f + 2, jp = j + 2;
      size_t qL = (size_t)jp * px + iL, qR = qL + 1;
      double un = V->unx[(size_t)j * (nx + 1) + f];
      fxf[(size_t)j * (nx + 1) + f] =
          face_flux(B, G->xcp, P->xe[f], qL - 1, qL, qR, qR + 1, iL, iR, 0, un, P->flux);
    }
  /* y-faces: jface = 0..ny between cells jface-1 and jface */
  for (int f = 0; f <= ny; ++f)
    for (int i = 0; i < nx; ++i) {
      int jL = f - 1 + 2, jR = f + 2, ip = i + 2;
      size_t qL = (size_t)jL * px + ip, qR = (size_t)jR * px + ip;
      double un = V->uny[(size_t)f * nx + i];
      fyf[(size_t)f * nx + i] =
          face_flux(B, G->ycp, P->ye[f], qL - px, qL, qR, qR + px, jL, jR, 1, un, P->flux);
    }
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      size_t c = (size_t)j * nx + i, ck = (size_t)k * nc + c;
      double e = E[ck], fxv = Fx[ck], fyv = Fy[ck];
      double dV = cell_volume(P, i, j);
      double Axp = area_x(P, i + 1, j), Axm = area_x(P, i, j), Ay = area_y(P, i);
      Flux3 xp = fxf[(size_t)j * (nx + 1) + i + 1], xm = fxf[(size_t)j * (nx + 1) + i];
      Flux3 yp = fyf[(size_t)(j + 1) * nx + i], ym = fyf[(size_t)j * nx + i];
      double divE = Axp * xp.e - Axm * xm.e + Ay * (yp.e - ym.e);
      double divX = Axp * xp.fx - Axm * xm.fx + Ay * (yp.fx - ym.fx);
      double divY = Axp * xp.fy - Axm * xm.fy + Ay * (yp.fy - ym.fy);
      const VelGrad *g = &V->grad[c];
      double work = D_colon_gradu(P, e, fxv, fyv, g) / C_LIGHT;
      double Es = e - ctdt / dV * divE - ctdt * work * e;
      double Xs = fxv - ctdt / dV * divX;
      double Ys = fyv - ctdt / dV * divY;
      if (P->geom == 1) {
        /* azimuthal (hoop) pressure: + D_phiphi E (A+ - A-)/dV */
        double Dxx, Dyy, Dxy, Dpp;
        eddington_tensor(e, fxv, fyv, &Dxx, &Dyy, &Dxy, &Dpp);
        Xs += ctdt * Dpp * e * (Axp - Axm) / dV;
      }
      /* causality: E >= 0 and |F| <= E at the cell centre */
      if (Es <= 0.0) { Es = 0.0; Xs = 0.0; Ys = 0.0; }
      else {
        double nF = hypot(Xs, Ys);
        if (nF > Es) { Xs *= Es / nF; Ys *= Es / nF; }
      }
      if (!source) { Eo[ck] = Es; Fxo[ck] = Xs; Fyo[ck] = Ys; continue; }
      /* implicit emission / absorption / destruction (BDF1, one substep) */
      double kE, aF, src;
      source_coeffs(P, k, c, &kE, &aF, &src);
      Eo[ck] = (Es + ctdt * src) / (1.0 + ctdt * kE);
      Fxo[ck] = Xs / (1.0 + ctdt * aF);
      Fyo[ck] = Ys / (1.0 + ctdt * aF);
    }
}

/* ------------------------------------------------------------------------ */
/* Frequency step helpers (Appendix A). */

/* e^{-m} (e^z - 1)/z for m >= max(z, 0); the value at z = 0 is e^{-m}. */
static double shifted_E1(double z, double m) {
  if (m < 700.0) return exp(-m) * (z == 0.0 ? 1.0 : expm1(z) / z);
  if (z == 0.0) return exp(-m);
  return (exp(z - m) - exp(-m)) / z;
}

/* Frequency flux through the interface between bin l (lower) and bin r:
 * F_nu = gr J_r - gl J_l.  Exponential scheme: gl = e^{-P_l+}/den,
 * gr = e^{P_r-}/den with den = (dl/Kl) chi^L(P_l+) - (dr/Kr) chi^R(P_r-),
 * P_l+ = Cl dl/Kl, P_r- = Cr dr/Kr.  Evaluated with numerator and
 * denominator multiplied by e^{-m}, m = max(-P_l+, P_r-, 0), so that nothing
 * overflows (an exact rewrite).  Cells without line opacity (K = 0) take the
 * K -> 0 limit: first-order upwind with rates max(-Cl,0), max(Cr,0). */
static void interface_rates(double Kl, double Cl, double dl, double Kr, double Cr,
                            double dr, double *gl, double *gr) {
  if (Kl == 0.0 || Kr == 0.0) {
    *gl = (Cl < 0.0) ? -Cl : 0.0;
    *gr = (Cr > 0.0) ? Cr : 0.0;
    return;
  }
  double A = -Cl * dl / Kl;
  double Bx = Cr * dr / Kr;
  double m = A > Bx ? A : Bx;
  if (m < 0.0) m = 0.0;
  double den = (dl / Kl) * shifted_E1(A, m) + (dr / Kr) * shifted_E1(Bx, m);
  *gl = exp(A - m) / den;
  *gr = exp(Bx - m) / den;
}

static void frequency_step_cell(const OracleProblem *P, const VelData *V, int i, int j, double *E,
                                double *Fx, double *Fy, const double *Ess,
                                const double *Xss, const double *Yss,
                                double *K, double *C, double *gl, double *gr,
                                long double *cp, long double *dp) {
  int nx = P->nx, nb = P->nb;
  size_t nc = (size_t)nx * P->ny, c = (size_t)j * nx + i;
  const VelGrad *g = &V->grad[c];
  double dnuD = P->dnuD[c];
  int cl = P->cls[c];
  for (int k = 0; k < nb; ++k) {
    size_t ck = (size_t)k * nc + c;
    double h = P->hbar[(size_t)cl * nb + k];
    K[k] = 0.5 * dnuD * dnuD * P->alpha[c] * h;
    double recoil = P->hkT[c] - 2.0 / P->nu_c[k];
    double Ck = 0.0;
    if (P->recoil) Ck += K[k] * recoil;
    if (P->doppler)
      Ck += P->nu_c[k] / C_LIGHT * D_colon_gradu(P, Ess[ck], Xss[ck], Yss[ck], g);
    C[k] = Ck;
  }
  /* interface k+1/2 between bins k and k+1; bin half-widths are dnu/2 */
  for (int k = 0; k + 1 < nb; ++k)
    interface_rates(K[k], C[k], 0.5 * P->dnu[k], K[k + 1], C[k + 1],
                    0.5 * P->dnu[k + 1], &gl[k], &gr[k]);
  /* BDF1:  (J^{n+1} - J^{em/abs}) / (c dt) = F+ J_{k+1} - F J_k + F- J_{k-1}
   * with F+_k = gr_{k+1/2}/dnu_k, F-_k = gl_{k-1/2}/dnu_k,
   * F_k = (gl_{k+1/2} + gr_{k-1/2})/dnu_k; zero flux at the grid ends.
   * Thomas algorithm in long double. */
  long double ct = (long double)P->c_tilde * (long double)P->dt;
  long double prev_c = 0.0L, prev_d = 0.0L;
  for (int k = 0; k < nb; ++k) {
    size_t ck = (size_t)k * nc + c;
    long double up = (k + 1 < nb) ? (long double)gl[k] : 0.0L;     /* out to k+1 */
    long double dn = (k > 0) ? (long double)gr[k - 1] : 0.0L;      /* out to k-1 */
    long double diag = 1.0L + ct * (up + dn) / (long double)P->dnu[k];
    long double sub = (k > 0) ? -ct * (long double)gl[k - 1] / (long double)P->dnu[k] : 0.0L;
    long double sup = (k + 1 < nb) ? -ct * (long double)gr[k] / (long double)P->dnu[k] : 0.0L;
    long double piv = diag - sub * prev_c;
    cp[k] = sup / piv;
    dp[k] = ((long double)Ess[ck] - sub * prev_d) / piv;
    prev_c = cp[k]; prev_d = dp[k];
  }
  long double x = 0.0L;
  for (int k = nb - 1; k >= 0; --k) {
    x = (k == nb - 1) ? dp[k] : dp[k] - cp[k] * x;
    size_t ck = (size_t)k * nc + c;
    double En = (double)x;
    double ratio = (Ess[ck] > 0.0) ? En / Ess[ck] : 0.0;
    E[ck] = En;
    Fx[ck] = Xss[ck] * ratio;
    Fy[ck] = Yss[ck] * ratio;
  }
}

/* ------------------------------------------------------------------------ */
/* Active bins (Section 2.2, active bins): the energy of bin k in the
 * volume is W_k = dnu_k sum_cells dV E_k (E = 4 pi J / c; constant factors
 * cancel in the ratio), and bin k is advected when W_k > active_frac sum_k W_k.
 * An empty state advects no bin. */
static void select_active_bins(const OracleProblem *P, const double *E, int *active) {
  int nx = P->nx, ny = P->ny, nb = P->nb;
  size_t nc = (size_t)nx * ny;
  double *W = (double *)malloc(sizeof(double) * nb);
  double total = 0.0;
  for (int k = 0; k < nb; ++k) {
    double s = 0.0;
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i)
        s += cell_volume(P, i, j) * E[(size_t)k * nc + (size_t)j * nx + i];
    W[k] = P->dnu[k] * s;
    total += W[k];
  }
  for (int k = 0; k < nb; ++k) active[k] = W[k] > P->active_frac * total;
  free(W);
}

/* ------------------------------------------------------------------------ */
/* Emission/absorption of one cell in substeps (Section 2.1, step 2).  A
 * substep of length h maps J. -> J.. = (J. + c h j)/(1 + c h kE) and
 * H. -> H.. = H./(1 + c h aF) in every bin; it is accepted when
 * |e.. - e.| < 0.1 (e. + e_floor), e = sum_k dnu_k E_k (the energy density),
 * e_floor = 4 pi J_floor / c with J_floor = 1e-15 erg cm^-2 s^-1 sr^-1, and
 * otherwise halved and redone.  After an accepted substep the next one tries
 * twice the length, clipped to the time left (a reading: the paper does not
 * say how the substep grows back).  A substep 2^-60 of the step, or the
 * 4096th attempt, is accepted as it is, so the loop always ends.
 * E, F (in/out, [nb] with stride nc) go from the post-transport to the
 * post-source state; f4 receives the step-averaged force, the sum over
 * substeps of (h/dt) sum_k dnu_k (F. - F..)/(c h), and its line part.  Since
 * F. - F.. = c h aF F.. exactly (the implicit update), each substep's force is
 * formed as sum_k dnu_k aF F.., free of the cancellation of the difference. */
#define SUB_MAX_ATTEMPTS 4096
static int source_substeps_cell(const OracleProblem *P, size_t c, size_t nc, double *E,
                                double *Fx, double *Fy, double *f4, double *Et,
                                double *margin) {
  int nb = P->nb;
  const double e_floor = 4.0 * ORACLE_PI * 1.0e-15 / C_LIGHT;
  const double dt = P->dt, ct = P->c_tilde;
  int cl = P->cls[c];
  double done = 0.0, h = dt;
  int accepted = 0;
  *margin = INFINITY;
  for (int q = 0; q < 4; ++q) f4[q] = 0.0;
  for (int attempt = 1; done < dt; ++attempt) {
    if (h > dt - done) h = dt - done;
    double e0 = 0.0, e1 = 0.0;
    for (int k = 0; k < nb; ++k) {
      size_t ck = (size_t)k * nc + c;
      double hb = P->hbar[(size_t)cl * nb + k];
      double kE = P->acabs[c] + P->pd[c] * P->alpha[c] * hb;
      double src = P->emis[c] * P->phi[(size_t)cl * nb + k] / C_LIGHT;
      Et[k] = (E[ck] + ct * h * src) / (1.0 + ct * h * kE);
      e0 += P->dnu[k] * E[ck];
      e1 += P->dnu[k] * Et[k];
    }
    double r = fabs(e1 - e0) / (e0 + e_floor);
    if (fabs(r / 0.1 - 1.0) < *margin) *margin = fabs(r / 0.1 - 1.0);
    int ok = fabs(e1 - e0) < 0.1 * (e0 + e_floor) || h <= ldexp(dt, -60) ||
             attempt >= SUB_MAX_ATTEMPTS;
    if (!ok) { h *= 0.5; continue; }
    for (int k = 0; k < nb; ++k) {
      size_t ck = (size_t)k * nc + c;
      double hb = P->hbar[(size_t)cl * nb + k];
      double aH = P->alpha[c] * hb, aF = aH + P->acF[c];
      double gx = Fx[ck] / (1.0 + ct * h * aF), gy = Fy[ck] / (1.0 + ct * h * aF);
      /* substep force sum_k dnu_k (F. - F..)/(c_tilde h) = sum_k dnu_k aF F..,
       * weighted by h/dt */
      double wx = P->dnu[k] * aF * gx * (h / dt), wy = P->dnu[k] * aF * gy * (h / dt);
      f4[0] += wx; f4[1] += wy;
      f4[2] += (aH / aF) * wx; f4[3] += (aH / aF) * wy;   /* line (gas) share */
      E[ck] = Et[k]; Fx[ck] = gx; Fy[ck] = gy;
    }
    done += h;
    ++accepted;
    h *= 2.0;
  }
  return accepted;
}

/* ------------------------------------------------------------------------ */
/* One full RT step.  E, Fx, Fy: state in/out [nb][ncell].
 * force: [4][ncell] = (f_x, f_y, f_x gas part, f_y gas part) of this step.
 * Ess, Xss, Yss: caller scratch of the state size (post-source state). */
int oracle_step(const OracleProblem *P, double *E, double *Fx, double *Fy,
                double *force, double *Ess, double *Xss, double *Yss) {
  int nx = P->nx, ny = P->ny, nb = P->nb;
  size_t nc = (size_t)nx * ny;
  Geometry G;
  build_geometry(P, &G);
  VelData V;
  build_velocity(P, &V);
  size_t npad = (size_t)(nx + 4) * (ny + 4);
  if (P->band && (P->active_frac > 0.0 || P->substep_rule)) return 1;
  int *active = (int *)malloc(sizeof(int) * nb);
  if (P->active_frac > 0.0) select_active_bins(P, E, active);
  else for (int k = 0; k < nb; ++k) active[k] = 1;
  if (P->active) memcpy(P->active, active, sizeof(int) * nb);
  /* (1)+(2): advection and emission/absorption, bins independent */
#pragma omp parallel
  {
    PadBin B;
    B.px = nx + 4;
    B.E = (double *)malloc(sizeof(double) * npad);
    B.fx = (double *)malloc(sizeof(double) * npad);
    B.fy = (double *)malloc(sizeof(double) * npad);
    B.aF = (double *)malloc(sizeof(double) * npad);
    Flux3 *fxf = (Flux3 *)malloc(sizeof(Flux3) * (size_t)(nx + 1) * ny);
    Flux3 *fyf = (Flux3 *)malloc(sizeof(Flux3) * (size_t)nx * (ny + 1));
#pragma omp for schedule(dynamic, 1)
    for (int k = 0; k < nb; ++k)
      advect_source_bin(P, &G, &V, k, active[k], !P->substep_rule, E, Fx, Fy, Ess, Xss, Yss,
                        &B, fxf, fyf);
    free(B.E); free(B.fx); free(B.fy); free(B.aF); free(fxf); free(fyf);
  }
  /* (2) with the substep rule: emission/absorption per cell, force with it */
  if (P->substep_rule) {
#pragma omp parallel
    {
      double *Et = (double *)malloc(sizeof(double) * nb);
#pragma omp for schedule(dynamic, 64)
      for (long c = 0; c < (long)nc; ++c) {
        double f4[4], mg;
        int n = source_substeps_cell(P, (size_t)c, nc, Ess, Xss, Yss, f4, Et, &mg);
        if (P->substeps) P->substeps[c] = n;
        if (P->sub_margin) P->sub_margin[c] = mg;
        for (int q = 0; q < 4; ++q) force[(size_t)q * nc + c] = f4[q];
      }
      free(Et);
    }
  }
  /* (3) radiation force density, f = sum_k dnu_k alpha_F,k F**_k (one
   * substep; the substep path formed it above) */
  long ncf = P->substep_rule ? 0 : (long)nc;
  if (P->band) {
    /* bands: f = sum_B kappa_F,B F**_B (band-integrated fluxes); the split
     * between gas and dust is not known here, the line part is left 0 */
#pragma omp parallel for schedule(static)
    for (long c = 0; c < (long)nc; ++c) {
      double sx = 0, sy = 0;
      for (int k = 0; k < nb; ++k) {
        size_t ck = (size_t)k * nc + c;
        sx += P->kflux[ck] * Xss[ck];
        sy += P->kflux[ck] * Yss[ck];
      }
      force[c] = sx; force[nc + c] = sy; force[2 * nc + c] = 0.0; force[3 * nc + c] = 0.0;
    }
    /* no frequency step: the post-source state is the new state */
    memcpy(E, Ess, sizeof(double) * nb * nc);
    memcpy(Fx, Xss, sizeof(double) * nb * nc);
    memcpy(Fy, Yss, sizeof(double) * nb * nc);
    ncf = 0;
  }
#pragma omp parallel for schedule(static)
  for (long c = 0; c < ncf; ++c) {
    double sx = 0, sy = 0, gx = 0, gy = 0;
    int cl = P->cls[c];
    for (int k = 0; k < nb; ++k) {
      size_t ck = (size_t)k * nc + c;
      double aH = P->alpha[c] * P->hbar[(size_t)cl * nb + k];
      double aF = aH + P->acF[c];
      sx += P->dnu[k] * aF * Xss[ck];
      sy += P->dnu[k] * aF * Yss[ck];
      gx += P->dnu[k] * aH * Xss[ck];
      gy += P->dnu[k] * aH * Yss[ck];
    }
    force[c] = sx; force[nc + c] = sy; force[2 * nc + c] = gx; force[3 * nc + c] = gy;
  }
  /* (4) frequency step, cells independent */
  long nfs = P->band ? 0 : (long)nc;
#pragma omp parallel
  {
    double *K = (double *)malloc(sizeof(double) * nb);
    double *Cc = (double *)malloc(sizeof(double) * nb);
    double *gl = (double *)malloc(sizeof(double) * nb);
    double *gr = (double *)malloc(sizeof(double) * nb);
    long double *cp = (long double *)malloc(sizeof(long double) * nb);
    long double *dp = (long double *)malloc(sizeof(long double) * nb);
#pragma omp for schedule(static)
    for (long c = 0; c < nfs; ++c)
      frequency_step_cell(P, &V, (int)(c % nx), (int)(c / nx), E, Fx, Fy, Ess, Xss, Yss,
                          K, Cc, gl, gr, cp, dp);
    free(K); free(Cc); free(gl); free(gr); free(cp); free(dp);
  }
  free(active);
  free_geometry(&G);
  free_velocity(&V);
  return 0;
}

/* Pieces exported for the oracle's own pin tests. */
void oracle_signal_speeds(double fx, double fy, int n, double *out2) {
  signal_speeds(fx, fy, n, &out2[0], &out2[1]);
}
void oracle_eddington(double E, double Fx, double Fy, double *out4) {
  eddington_tensor(E, Fx, Fy, &out4[0], &out4[1], &out4[2], &out4[3]);
}
void oracle_interface_rates(double Kl, double Cl, double dl, double Kr, double Cr,
                            double dr, double *out2) {
  interface_rates(Kl, Cl, dl, Kr, Cr, dr, &out2[0], &out2[1]);
}
int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of the following parallel regions (n >= 1); changes no arithmetic. */
void oracle_set_num_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
