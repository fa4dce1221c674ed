// Hot-path kernels of the M1 Lyman-alpha step (gfx950, wave64).
//
//   advect_source : Section 2.1 steps 1 and 2 for a run of bins of one cell
//                   per lane: MinMod reconstruction of E and f, Levermore
//                   closure, GLF flux (HLL with signal speeds +-c_tilde)
//                   blended with the diffusion flux by eps(tau), upwind
//                   velocity advection, work term, hoop pressure (R, z),
//                   causality clamp, implicit emission/absorption (BDF1).
//   freq_step     : Section 2.3 force density and Appendix A frequency step
//                   for all bins of one cell per lane: exponential-scheme
//                   interface rates, subtraction-free elimination of the
//                   tridiagonal system in photon-number variables, H rescale.
//   residual      : deterministic FP64 norms ||E^{n+1} - E^n||, ||E^{n+1}||.
#include "m1_kernels.h"

namespace m1 {

// ----------------------------------------------------------- state loading
// Value of (E, f_x, f_y) of cell (ii, jj) of bin offset koff, with ghost
// cells: vacuum -> E = f = 0; reflecting -> mirror image with the normal
// component of f negated.  At most one of ii, jj is out of range.
template <typename R>
__device__ __forceinline__ void load_ef(const GridArgs<R>& a, size_t koff, int ii, int jj,
                                        R& e, R& fx, R& fy) {
  int si = ii, sj = jj;
  R sx = R(1), sy = R(1);
  if (ii < 0 || ii >= a.nx) {
    int side = ii < 0 ? 0 : 1;
    if (a.bc[side] != kReflect) { e = fx = fy = R(0); return; }
    si = ii < 0 ? -1 - ii : 2 * a.nx - 1 - ii;
    sx = R(-1);
  } else if (jj < 0 || jj >= a.ny) {
    int side = jj < 0 ? 2 : 3;
    if (a.bc[side] != kReflect) { e = fx = fy = R(0); return; }
    sj = jj < 0 ? -1 - jj : 2 * a.ny - 1 - jj;
    sy = R(-1);
  }
  size_t q = koff + (size_t)sj * a.nx + si;
  e = a.E[q];
  reduced_flux(e, a.Fx[q], a.Fy[q], fx, fy);
  fx *= sx;
  fy *= sy;
}

// Static opacity data of a neighbour (mirror cell at reflecting boundaries;
// alpha_F = 0 in vacuum ghosts).
template <typename R>
struct NbrOpacity {
  int cls;
  R alpha, acF;
};

template <typename R>
__device__ __forceinline__ NbrOpacity<R> nbr_opacity(const GridArgs<R>& a, int ii, int jj) {
  NbrOpacity<R> o;
  int si = ii, sj = jj;
  if (ii < 0 || ii >= a.nx) {
    int side = ii < 0 ? 0 : 1;
    if (a.bc[side] != kReflect) { o.cls = 0; o.alpha = R(0); o.acF = R(0); return o; }
    si = ii < 0 ? -1 - ii : 2 * a.nx - 1 - ii;
  } else if (jj < 0 || jj >= a.ny) {
    int side = jj < 0 ? 2 : 3;
    if (a.bc[side] != kReflect) { o.cls = 0; o.alpha = R(0); o.acF = R(0); return o; }
    sj = jj < 0 ? -1 - jj : 2 * a.ny - 1 - jj;
  }
  size_t c = (size_t)sj * a.nx + si;
  o.cls = a.cls[c];
  o.alpha = a.alpha[c];
  o.acF = a.acF[c];
  return o;
}

template <typename R>
struct Flux3 {
  R e, x, y;
};

// Flux of (E, F_x, F_y) through one face with normal n (0: x, 1: y).
// Cells along the normal: LL, L | face | R, RR (values e*, fx*, fy*).
// iLL = 1/(c_L - c_LL), iLR = 1/(c_R - c_L), iRR = 1/(c_RR - c_R) are inverse
// centroid distances; hL = x_f - c_L > 0, hR = x_f - c_R < 0.
template <typename R, int N>
__device__ __forceinline__ Flux3<R> face_flux(R eLL, R xLL, R yLL, R eL, R xL, R yL,
                                              R eR, R xR, R yR, R eRR, R xRR, R yRR,
                                              R iLL, R iLR, R iRR, R hL, R hR,
                                              R aFL, R aFR, R un_c) {
  // MinMod slopes of E, f_x, f_y on both sides and reconstructed face states
  R dE = (eR - eL) * iLR, dX = (xR - xL) * iLR, dY = (yR - yL) * iLR;
  R EL = eL + minmod((eL - eLL) * iLL, dE) * hL;
  R fxL = xL + minmod((xL - xLL) * iLL, dX) * hL;
  R fyL = yL + minmod((yL - yLL) * iLL, dY) * hL;
  R ER = eR + minmod(dE, (eRR - eR) * iRR) * hR;
  R fxR = xR + minmod(dX, (xRR - xR) * iRR) * hR;
  R fyR = yR + minmod(dY, (yRR - yR) * iRR) * hR;
  // causality at the interface: |f| > 1 is scaled back to 1
  R nL = fxL * fxL + fyL * fyL, nR = fxR * fxR + fyR * fyR;
  if (nL > R(1)) { R s = R(1) / sqrt(nL); fxL *= s; fyL *= s; }
  if (nR > R(1)) { R s = R(1) / sqrt(nR); fxR *= s; fyR *= s; }
  Eddington<R> DL = closure_f(fxL, fyL), DR = closure_f(fxR, fyR);
  R FxL = fxL * EL, FyL = fyL * EL, FxR = fxR * ER, FyR = fyR * ER;
  R PxL, PyL, PxR, PyR;       // row n of the pressure tensor, P = D E
  if (N == 0) { PxL = DL.xx * EL; PyL = DL.xy * EL; PxR = DR.xx * ER; PyR = DR.xy * ER; }
  else        { PxL = DL.xy * EL; PyL = DL.yy * EL; PxR = DR.xy * ER; PyR = DR.yy * ER; }
  // flux optical depth between the centroids and the blend eps(tau)
  R tau = aFL * hL - aFR * hR;
  R inv = R(1) / (R(0.2) + tau + tau * tau);
  R eps = (R(0.2) + tau) * inv;
  R dco = tau * inv * R(1.0 / 3.0);     // (1 - eps) / (3 tau)
  R FnL = (N == 0) ? FxL : FyL, FnR = (N == 0) ? FxR : FyR;
  Flux3<R> r;
  r.e = eps * (R(0.5) * (FnL + FnR) - R(0.5) * (ER - EL)) - dco * (eR - eL);
  r.x = R(0.5) * (PxL + PxR) - eps * R(0.5) * (FxR - FxL);
  r.y = R(0.5) * (PyL + PyR) - eps * R(0.5) * (FyR - FyL);
  // upwind advection by the face velocity with the upstream reconstruction
  if (un_c > R(0)) { r.e += un_c * EL; r.x += un_c * FxL; r.y += un_c * FyL; }
  else if (un_c < R(0)) { r.e += un_c * ER; r.x += un_c * FxR; r.y += un_c * FyR; }
  return r;
}

// ---------------------------------------------------------------- K2
// Block: 64 x 4 lanes (x fastest, coalesced rows); each lane walks BK bins of
// one cell so the cell's static data is loaded once per BK bins.
template <typename R, int BK>
__global__ __launch_bounds__(256) void k_advect_source(GridArgs<R> a) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  const int j = blockIdx.y * 4 + threadIdx.y;
  const int k0 = blockIdx.z * BK;
  if (i >= a.nx || j >= a.ny) return;
  const int nx = a.nx;
  const size_t nc = (size_t)nx * a.ny;
  const size_t c = (size_t)j * nx + i;
  const R inv_c = R(1.0 / kC);

  // static data of the cell and its four face neighbours
  const int clsC = a.cls[c];
  const R alC = a.alpha[c], acFC = a.acF[c], acabsC = a.acabs[c], pdaC = a.pda[c];
  const R emC = a.em[c];
  const NbrOpacity<R> oW = nbr_opacity(a, i - 1, j), oE = nbr_opacity(a, i + 1, j);
  const NbrOpacity<R> oS = nbr_opacity(a, i, j - 1), oN = nbr_opacity(a, i, j + 1);
  const R gxx = a.grad[c], gyy = a.grad[nc + c], gxy = a.grad[2 * nc + c],
          gpp = a.grad[3 * nc + c];
  const R uW = a.ufx[(size_t)j * (nx + 1) + i] * inv_c;
  const R uE = a.ufx[(size_t)j * (nx + 1) + i + 1] * inv_c;
  const R uS = a.ufy[c] * inv_c;
  const R uN = a.ufy[c + nx] * inv_c;
  // geometry (x: column index + 2; y: row index + 2)
  const R xi_m = a.xidl[i + 1], xi_c = a.xidl[i + 2], xi_p = a.xidl[i + 3], xi_pp = a.xidl[i + 4];
  const R xhp_W = a.xhp[i + 1], xhm_C = a.xhm[i + 2], xhp_C = a.xhp[i + 2], xhm_E = a.xhm[i + 3];
  const R yi_m = a.yidl[j + 1], yi_c = a.yidl[j + 2], yi_p = a.yidl[j + 3], yi_pp = a.yidl[j + 4];
  const R yhp_S = a.yhp[j + 1], yhm_C = a.yhm[j + 2], yhp_C = a.yhp[j + 2], yhm_N = a.yhm[j + 3];
  const R cxm = a.cxm[i], cxp = a.cxp[i], chp = a.chp[i], cy = a.cy[j];
  const R ctdt = a.ctdt, ctdt_c = a.ctdt_c;
  const bool moving = (gxx != R(0)) || (gyy != R(0)) || (gxy != R(0)) || (gpp != R(0));

  const int kend = min(k0 + BK, a.nb);
  for (int k = k0; k < kend; ++k) {
    const size_t koff = (size_t)k * nc;
    const R* hb = a.hbar;
    const int nb = a.nb;
    // opacities of this bin
    const R hC = hb[(size_t)clsC * nb + k];
    const R aFC = alC * hC + acFC;
    const R aFW = oW.alpha * hb[(size_t)oW.cls * nb + k] + oW.acF;
    const R aFE = oE.alpha * hb[(size_t)oE.cls * nb + k] + oE.acF;
    const R aFS = oS.alpha * hb[(size_t)oS.cls * nb + k] + oS.acF;
    const R aFN = oN.alpha * hb[(size_t)oN.cls * nb + k] + oN.acF;
    // stencil: centre, and two cells each way along x and y
    R eC, xC, yC;
    const R EC = a.E[koff + c], FXC = a.Fx[koff + c], FYC = a.Fy[koff + c];
    eC = EC;
    reduced_flux(EC, FXC, FYC, xC, yC);
    R eWW, xWW, yWW, eW, xW, yW, eE, xE, yE, eEE, xEE, yEE;
    load_ef(a, koff, i - 2, j, eWW, xWW, yWW);
    load_ef(a, koff, i - 1, j, eW, xW, yW);
    load_ef(a, koff, i + 1, j, eE, xE, yE);
    load_ef(a, koff, i + 2, j, eEE, xEE, yEE);
    R eSS, xSS, ySS, eS, xS, yS, eN, xN, yN, eNN, xNN, yNN;
    load_ef(a, koff, i, j - 2, eSS, xSS, ySS);
    load_ef(a, koff, i, j - 1, eS, xS, yS);
    load_ef(a, koff, i, j + 1, eN, xN, yN);
    load_ef(a, koff, i, j + 2, eNN, xNN, yNN);
    // four face fluxes
    Flux3<R> fW = face_flux<R, 0>(eWW, xWW, yWW, eW, xW, yW, eC, xC, yC, eE, xE, yE,
                                  xi_m, xi_c, xi_p, xhp_W, xhm_C, aFW, aFC, uW);
    Flux3<R> fE = face_flux<R, 0>(eW, xW, yW, eC, xC, yC, eE, xE, yE, eEE, xEE, yEE,
                                  xi_c, xi_p, xi_pp, xhp_C, xhm_E, aFC, aFE, uE);
    Flux3<R> fS = face_flux<R, 1>(eSS, xSS, ySS, eS, xS, yS, eC, xC, yC, eN, xN, yN,
                                  yi_m, yi_c, yi_p, yhp_S, yhm_C, aFS, aFC, uS);
    Flux3<R> fN = face_flux<R, 1>(eS, xS, yS, eC, xC, yC, eN, xN, yN, eNN, xNN, yNN,
                                  yi_c, yi_p, yi_pp, yhp_C, yhm_N, aFC, aFN, uN);
    // conservative update, work term and hoop pressure
    Eddington<R> D = closure_state(EC, FXC, FYC);
    R Es = EC - (cxp * fE.e - cxm * fW.e + cy * (fN.e - fS.e));
    R Xs = FXC - (cxp * fE.x - cxm * fW.x + cy * (fN.x - fS.x));
    R Ys = FYC - (cxp * fE.y - cxm * fW.y + cy * (fN.y - fS.y));
    if (moving) Es -= ctdt_c * (D.xx * gxx + D.yy * gyy + D.xy * gxy + D.pp * gpp) * EC;
    Xs += chp * D.pp * EC;
    // causality: E >= 0, |F| <= E
    if (Es <= R(0)) { Es = R(0); Xs = R(0); Ys = R(0); }
    else {
      R n2 = Xs * Xs + Ys * Ys;
      if (n2 > Es * Es) { R s = Es / sqrt(n2); Xs *= s; Ys *= s; }
    }
    // implicit emission / absorption / destruction
    const R src = emC * a.phi[(size_t)clsC * nb + k];
    const R kE = acabsC + pdaC * hC;
    a.Eo[koff + c] = (Es + ctdt * src) / (R(1) + ctdt * kE);
    const R dF = R(1) / (R(1) + ctdt * aFC);
    a.Fxo[koff + c] = Xs * dF;
    a.Fyo[koff + c] = Ys * dF;
  }
}

// ---------------------------------------------------------------- K3
// e^{-m} (e^z - 1)/z for m >= max(z, 0) without overflow.
template <typename T>
__device__ __forceinline__ T shifted_E1(T z, T m) {
  const T lim = sizeof(T) == 8 ? T(700) : T(80);
  if (m < lim) return exp(-m) * (z == T(0) ? T(1) : expm1(z) / z);
  if (z == T(0)) return exp(-m);
  return (exp(z - m) - exp(-m)) / z;
}

// Exponential-scheme interface between bins l < r: frequency flux
// F = gr J_r - gl J_l with gl = e^{-Pl}/den, gr = e^{Pr}/den,
// den = (dl/Kl)(1 - e^{-Pl})/Pl + (dr/Kr)(e^{Pr} - 1)/Pr, Pl = Cl dl/Kl,
// Pr = Cr dr/Kr, all scaled by e^{-m}, m = max(-Pl, Pr, 0).  Without line
// opacity (K = 0) the scheme's upwind limit.
template <typename T>
__device__ __forceinline__ void interface_rates(T Kl, T Cl, T dl, T Kr, T Cr, T dr,
                                                T& gl, T& gr) {
  if (Kl == T(0) || Kr == T(0)) {
    gl = Cl < T(0) ? -Cl : T(0);
    gr = Cr > T(0) ? Cr : T(0);
    return;
  }
  T ql = dl / Kl, qr = dr / Kr;
  T A = -Cl * ql, B = Cr * qr;
  T m = A > B ? A : B;
  if (m < T(0)) m = T(0);
  T den = ql * shifted_E1(A, m) + qr * shifted_E1(B, m);
  T iden = T(1) / den;
  gl = exp(A - m) * iden;
  gr = exp(B - m) * iden;
}

// Frequency step and force of one cell.  R: storage type, T: arithmetic type.
//
// Photon-number variables y_k = dnu_k E_k.  The BDF1 system is
//   (1 + a_k + b_k) y_k - b_{k+1} y_{k+1} - a_{k-1} y_{k-1} = y_k^{old},
// a_k = ctdt gl_{k+1/2}/dnu_k (to k+1), b_k = ctdt gr_{k-1/2}/dnu_k (to k-1),
// whose columns sum to one (the step conserves photons).  Gaussian
// elimination keeps every quantity a sum or product of positive numbers:
// pivot p_k = s_k + a_k with s_k = 1 + b_k s_{k-1}/p_{k-1}, right-hand side
// d_k = y_k + a_{k-1} d_{k-1}/p_{k-1}, back substitution
// y_k = d_k/p_k + (b_{k+1}/p_k) y_{k+1}.  No subtraction, so the relative
// error stays O(N_nu eps) however stiff the cell is.
template <typename R, typename T>
__device__ void freq_cell(const GridArgs<R>& a, size_t c) {
  const size_t nc = (size_t)a.nx * a.ny;
  const int nb = a.nb;
  const int cl = a.cls[c];
  const T al = (T)a.alpha[c];
  const T acF = (T)a.acF[c];
  const T gxx = (T)a.grad[c], gyy = (T)a.grad[nc + c], gxy = (T)a.grad[2 * nc + c],
          gpp = (T)a.grad[3 * nc + c];
  const T dd = (T)a.dD2h[cl] * al;
  const T hkT = (T)a.hkT[cl];
  const T ctdt = (T)a.ctdt;
  const R* hb = a.hbar + (size_t)cl * nb;
  const bool use_recoil = a.recoil != 0;
  const bool use_doppler = a.doppler != 0 &&
      ((gxx != T(0)) || (gyy != T(0)) || (gxy != T(0)) || (gpp != T(0)));

  double fx = 0.0, fy = 0.0, gx = 0.0, gy = 0.0;
  auto coeffs = [&](int k, T& K, T& C) {
    const size_t q = (size_t)k * nc + c;
    const R e = a.Eo[q], X = a.Fxo[q], Y = a.Fyo[q];
    const T h = (T)hb[k];
    K = dd * h;
    C = T(0);
    if (use_recoil) C += K * (hkT - (T)a.two_nu[k]);
    if (use_doppler) {
      Eddington<T> D = closure_state<T>((T)e, (T)X, (T)Y);
      C += (T)a.nu_c[k] * (D.xx * gxx + D.yy * gyy + D.xy * gxy + D.pp * gpp);
    }
    // force density: sum_k dnu_k alpha_F,k F**_k (and the line part)
    const double dn = a.dnu[k];
    const double aH = (double)al * (double)h;
    const double aF = aH + (double)acF;
    fx += dn * aF * (double)X;
    fy += dn * aF * (double)Y;
    gx += dn * aH * (double)X;
    gy += dn * aH * (double)Y;
  };

  T Kc, Cc;
  coeffs(0, Kc, Cc);
  T s_prev = T(1), p_prev = T(1), d_prev = T(0), a_prev = T(0);
  T b_k = T(0);             // rate of bin k toward k-1 (zero at the lower end)
  for (int k = 0; k < nb; ++k) {
    T a_k = T(0), b_next = T(0);
    const T dnk = (T)a.dnu[k];
    if (k + 1 < nb) {
      T Kn, Cn;
      coeffs(k + 1, Kn, Cn);
      const T dnn = (T)a.dnu[k + 1];
      T gl, gr;
      interface_rates<T>(Kc, Cc, T(0.5) * dnk, Kn, Cn, T(0.5) * dnn, gl, gr);
      a_k = ctdt * gl / dnk;
      b_next = ctdt * gr / dnn;
      Kc = Kn;
      Cc = Cn;
    }
    const size_t q = (size_t)k * nc + c;
    const T y = dnk * (T)a.Eo[q];
    T s, d;
    if (k == 0) { s = T(1); d = y; }
    else {
      const T r = T(1) / p_prev;
      s = T(1) + b_k * s_prev * r;
      d = y + a_prev * d_prev * r;
    }
    const T p = s + a_k;
    const T ip = T(1) / p;
    a.zs[q] = (R)(d * ip);
    a.ws[q] = (R)(b_next * ip);
    s_prev = s; p_prev = p; d_prev = d; a_prev = a_k; b_k = b_next;
  }
  // back substitution and F rescale (F^{n+1} = F** E^{n+1}/E**)
  T y = T(0);
  for (int k = nb - 1; k >= 0; --k) {
    const size_t q = (size_t)k * nc + c;
    y = (T)a.zs[q] + (T)a.ws[q] * y;
    const T En = y / (T)a.dnu[k];
    const T Eo = (T)a.Eo[q];
    // F^{n+1} = (F**/E**) E^{n+1}, with |F**/E**| <= 1
    T fxo, fyo;
    reduced_flux<T>(Eo, (T)a.Fxo[q], (T)a.Fyo[q], fxo, fyo);
    a.Eo[q] = (R)En;
    a.Fxo[q] = (R)(fxo * En);
    a.Fyo[q] = (R)(fyo * En);
  }
  a.force[c] = fx;
  a.force[nc + c] = fy;
  a.force[2 * nc + c] = gx;
  a.force[3 * nc + c] = gy;
}

template <typename R>
__global__ __launch_bounds__(256) void k_freq(GridArgs<R> a) {
  const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (size_t)a.nx * a.ny) return;
  if (sizeof(R) == 8 || a.island[c]) freq_cell<R, double>(a, c);
  else freq_cell<R, float>(a, c);
}

// ---------------------------------------------------------------- K4
// Block partial sums of (E1 - E0)^2 and E1^2 in FP64, fixed order.
template <typename R>
__global__ __launch_bounds__(256) void k_residual(const R* __restrict__ E0,
                                                  const R* __restrict__ E1, size_t n,
                                                  double* __restrict__ partial) {
  __shared__ double s0[256], s1[256];
  double a0 = 0.0, a1 = 0.0;
  for (size_t q = (size_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (size_t)gridDim.x * 256) {
    double e1 = (double)E1[q], d = e1 - (double)E0[q];
    a0 += d * d;
    a1 += e1 * e1;
  }
  s0[threadIdx.x] = a0;
  s1[threadIdx.x] = a1;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s0[threadIdx.x] += s0[threadIdx.x + w];
      s1[threadIdx.x] += s1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = s0[0];
    partial[2 * blockIdx.x + 1] = s1[0];
  }
}

__global__ void k_residual_final(const double* __restrict__ partial, int nblk,
                                 double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double a0 = 0.0, a1 = 0.0;
  for (int b = 0; b < nblk; ++b) { a0 += partial[2 * b]; a1 += partial[2 * b + 1]; }
  out[0] = a0;
  out[1] = a1;
}

// ------------------------------------------------------- copies with scale
template <typename S, typename D>
__global__ void k_scale_copy(const S* __restrict__ src, D* __restrict__ dst, size_t n, int e2) {
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (size_t)gridDim.x * blockDim.x)
    dst[q] = (D)ldexp((double)src[q], e2);
}

__global__ void k_force_out(const double* __restrict__ force, size_t nc, int e2,
                            double* fx, double* fy, double* gx, double* gy) {
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < nc;
       c += (size_t)gridDim.x * blockDim.x) {
    if (fx) fx[c] = ldexp(force[c], e2);
    if (fy) fy[c] = ldexp(force[nc + c], e2);
    if (gx) gx[c] = ldexp(force[2 * nc + c], e2);
    if (gy) gy[c] = ldexp(force[3 * nc + c], e2);
  }
}

// ------------------------------------------------------------ launchers
constexpr int kBK = 8;

template <typename R>
hipError_t launch_advect(const GridArgs<R>& a, hipStream_t s) {
  dim3 blk(64, 4, 1);
  dim3 grd((a.nx + 63) / 64, (a.ny + 3) / 4, (a.nb + kBK - 1) / kBK);
  hipLaunchKernelGGL((k_advect_source<R, kBK>), grd, blk, 0, s, a);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_freq(const GridArgs<R>& a, hipStream_t s) {
  size_t nc = (size_t)a.nx * a.ny;
  hipLaunchKernelGGL((k_freq<R>), dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_step(const GridArgs<R>& a, hipStream_t s) {
  hipError_t e = launch_advect(a, s);
  if (e != hipSuccess) return e;
  return launch_freq(a, s);
}

template <typename R>
hipError_t launch_residual(const R* E0, const R* E1, size_t n, double* partial, int nblk,
                           double* out, hipStream_t s) {
  hipLaunchKernelGGL((k_residual<R>), dim3(nblk), dim3(256), 0, s, E0, E1, n, partial);
  hipLaunchKernelGGL(k_residual_final, dim3(1), dim3(64), 0, s, partial, nblk, out);
  return hipGetLastError();
}

template <typename S, typename D>
hipError_t launch_scale_copy(const S* src, D* dst, size_t n, int e2, hipStream_t s) {
  unsigned g = (unsigned)std::min<size_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL((k_scale_copy<S, D>), dim3(g ? g : 1), dim3(256), 0, s, src, dst, n, e2);
  return hipGetLastError();
}

hipError_t launch_force_out(const double* force, size_t nc, int e2, double* fx, double* fy,
                            double* gx, double* gy, hipStream_t s) {
  unsigned g = (unsigned)std::min<size_t>((nc + 255) / 256, 65536);
  hipLaunchKernelGGL(k_force_out, dim3(g ? g : 1), dim3(256), 0, s, force, nc, e2, fx, fy, gx, gy);
  return hipGetLastError();
}

template hipError_t launch_step<float>(const GridArgs<float>&, hipStream_t);
template hipError_t launch_advect<float>(const GridArgs<float>&, hipStream_t);
template hipError_t launch_advect<double>(const GridArgs<double>&, hipStream_t);
template hipError_t launch_freq<float>(const GridArgs<float>&, hipStream_t);
template hipError_t launch_freq<double>(const GridArgs<double>&, hipStream_t);
template hipError_t launch_step<double>(const GridArgs<double>&, hipStream_t);
template hipError_t launch_residual<float>(const float*, const float*, size_t, double*, int, double*, hipStream_t);
template hipError_t launch_residual<double>(const double*, const double*, size_t, double*, int, double*, hipStream_t);
template hipError_t launch_scale_copy<float, double>(const float*, double*, size_t, int, hipStream_t);
template hipError_t launch_scale_copy<double, float>(const double*, float*, size_t, int, hipStream_t);
template hipError_t launch_scale_copy<double, double>(const double*, double*, size_t, int, hipStream_t);

}  // namespace m1
