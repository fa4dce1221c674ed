// Hot-path kernels of the M1 Lyman-alpha step (gfx950, wave64).
//
//   advect_source : Section 2.1 steps 1 and 2; a block per 32 x 16 tile and
//                   run of bins, two cells per lane: MinMod reconstruction of
//                   E and f, Levermore closure, GLF flux (HLL with signal
//                   speeds +-c_tilde) blended with the diffusion flux by
//                   eps(tau), upwind velocity advection, work term, hoop
//                   pressure (R, z), causality clamp, implicit
//                   emission/absorption (BDF1).
//   freq_step     : Section 2.3 force density and Appendix A frequency step
//                   for all bins of one cell per lane: exponential-scheme
//                   interface rates, subtraction-free elimination of the
//                   tridiagonal system in photon-number variables.  The H
//                   rescale F -> F E^{n+1}/E** keeps f = F/E, which is what
//                   the state stores, so only E is rewritten.
//   step_fused    : both in one kernel, a block per tile and all bins (a
//                   batch tile variant).
//   freq_sub      : the frequency step with the emission/absorption of the
//                   step in substeps under the 10 % energy rule (Section 2.1,
//                   step 2; optional).
//   bin_energy,   : the active-bin selection of Section 2.1 (optional):
//   bin_select      per-bin energies in double, flags of the advected bins.
//   band_step     : the advection + emission/absorption kernel for a grid
//                   of broad bands (Section 2.5): per band and cell
//                   opacities and emission, force summed over the bands,
//                   no frequency step.
//   residual      : deterministic FP64 norms ||E^{n+1} - E^n||, ||E^{n+1}||.
#include "m1_kernels.h"

namespace m1 {

template <typename R>
struct Flux3 {
  R e, x, y;
};

// Signal speeds of the M1 system across a face, in units of c_tilde: the
// smallest and largest eigenvalues of the Jacobian of the face flux
// (F_n, P_nn, P_nt) with respect to (E, F_n, F_t), for the reduced flux of
// normal and tangential components (fn, ft), |f| <= 1 (the eigenvalues do not
// depend on the order of the flux components, so local face coordinates
// serve both directions).  With D = iso I + g f (x) f (the Levermore closure
// in the form of closure_f; q = f^2, s = sqrt(4 - 3 q), iso = (s - 1)/3,
// g = 3/(2 + s), d iso/dq = -1/(2 s), dg/dq = 9/(2 s (2 + s)^2)) and P = D E
// homogeneous of degree one, the Jacobian is
//   [ 0    1    0  ]
//   [ a1   b1   c1 ]   b1 = dD_nn/df_n, c1 = dD_nn/df_t, a1 = D_nn - fn b1 - ft c1,
//   [ a2   b2   c2 ]   b2 = dD_nt/df_n, c2 = dD_nt/df_t, a2 = D_nt - fn b2 - ft c2,
// whose characteristic polynomial is
//   lambda^3 - (b1 + c2) lambda^2 + (b1 c2 - b2 c1 - a1) lambda + (a1 c2 - a2 c1).
// Its three real roots (the system is hyperbolic) come from the
// trigonometric solution of the depressed cubic, in double for either
// storage precision.  As |f| -> 1 they merge at fn, and computed roots then
// carry errors up to the cube root of the rounding.
__device__ __forceinline__ void m1_signal_speeds(double fn, double ft, double& lo, double& hi) {
  double q = fn * fn + ft * ft;
  q = q < 1.0 ? q : 1.0;
  const double s = fsqrt(4.0 - 3.0 * q);            // in [1, 2]
  const double is = frcp(s), ip = frcp(2.0 + s);
  const double iso = (s - 1.0) * (1.0 / 3.0), g = 3.0 * ip;
  const double diso = -0.5 * is, dg = 4.5 * is * ip * ip;
  const double fn2 = fn * fn, ft2 = ft * ft;
  const double b1 = 2.0 * fn * (diso + dg * fn2 + g);
  const double c1 = 2.0 * ft * (diso + dg * fn2);
  const double b2 = ft * (2.0 * dg * fn2 + g);
  const double c2 = fn * (2.0 * dg * ft2 + g);
  const double a1 = (iso + g * fn2) - fn * b1 - ft * c1;
  const double a2 = g * fn * ft - fn * b2 - ft * c2;
  // lambda^3 + A lambda^2 + B lambda + C
  const double A = -(b1 + c2), B = b1 * c2 - b2 * c1 - a1, C = a1 * c2 - a2 * c1;
  const double p = B - A * A * (1.0 / 3.0);
  const double r = A * A * A * (2.0 / 27.0) - A * B * (1.0 / 3.0) + C;
  const double shift = -A * (1.0 / 3.0);
  if (p >= 0.0) {                // a triple root (p = 0 up to rounding)
    lo = hi = shift;
    return;
  }
  const double m2 = 2.0 * sqrt(-p * (1.0 / 3.0));
  double arg = 3.0 * r / (p * m2);                    // cos(3 theta)
  arg = arg > 1.0 ? 1.0 : (arg < -1.0 ? -1.0 : arg);
  const double th = acos(arg) * (1.0 / 3.0);
  hi = shift + m2 * cos(th);
  lo = shift + m2 * cos(th - 4.1887902047863909846);   // theta - 4 pi / 3
}

// Flux of (E, F_x, F_y) through one face with normal n (0: x, 1: y), from
// the reconstructed states on its two sides (EL, fxL, fyL | ER, fxR, fyR),
// the difference of the cell values dEc = e_R - e_L (diffusion term), the
// centroid distances hL = x_f - c_L > 0 and hR = x_f - c_R < 0, the flux
// opacities of the two cells and the face-normal velocity over c.
// The GLF flux is formed from half the pressure rows and half of eps (both
// exact halvings):  F_E = (eps/2) (F_nL + F_nR - (E_R - E_L)) - dco dEc,
// F_F = (P_L + P_R)/2 - (eps/2) (F_R - F_L).
// EIG: HLL with the M1 signal speeds (m1_signal_speeds, Davis estimates over
// the two states, clipped at zero) in place of -1, +1: the central part
// (sR G_L - sL G_R)/(sR - sL) and the dissipation sL sR (U_R - U_L)/(sR - sL),
// blended with eps as the GLF flux is; where both speeds are zero no wave
// crosses the face and the flux is the mean of the two states' fluxes.
template <typename R>
struct FaceSide {
  R Fx, Fy;       // F = f E
  R hPx, hPy;     // half of row n of the pressure tensor P = D E
};

// One side of a face: F and half of row n of P = D E, with
// D = iso I + g f (x) f (closure_parts), f2 = |f|^2 <= 1 up to rounding.
template <typename R, int N>
__device__ __forceinline__ FaceSide<R> face_side(R E, R fx, R fy, R f2) {
  FaceSide<R> o;
  const R s = fsqrt(R(4) - R(3) * clamp_unit(f2));
  const R hg = frcp(s * R(2.0 / 3.0) + R(4.0 / 3.0));      // g / 2
  const R e6 = E * R(1.0 / 6.0);
  const R hiE = fma(s, e6, -e6);                           // iso E / 2 = (s - 1) E / 6
  o.Fx = fx * E;
  o.Fy = fy * E;
  const R t = hg * (N == 0 ? o.Fx : o.Fy);                 // g F_n / 2
  o.hPx = N == 0 ? t * fx + hiE : t * fx;
  o.hPy = N == 0 ? t * fy : t * fy + hiE;
  return o;
}

template <typename R, int N, bool EIG = false>
__device__ __forceinline__ Flux3<R> face_flux(R EL, R fxL, R fyL, R ER, R fxR, R fyR, R dEc,
                                              R hL, R hR, R aFL, R aFR, R un_c) {
  // causality at the interface: |f| > 1 is scaled back to 1
  R nL = fxL * fxL + fyL * fyL, nR = fxR * fxR + fyR * fyR;
  if (nL > R(1) || nR > R(1)) [[unlikely]] {    // rare: one branch for both sides
    const R sL = nL > R(1) ? frsq(nL) : R(1), sR = nR > R(1) ? frsq(nR) : R(1);
    fxL *= sL; fyL *= sL; fxR *= sR; fyR *= sR;
    nL = fxL * fxL + fyL * fyL;
    nR = fxR * fxR + fyR * fyR;
  }
  const FaceSide<R> L = face_side<R, N>(EL, fxL, fyL, nL);
  const FaceSide<R> Q = face_side<R, N>(ER, fxR, fyR, nR);
  // flux optical depth between the centroids and the blend eps(tau)
  const R tau = aFL * hL - aFR * hR;
  const R t02 = tau + R(0.2);
  const R inv = frcp(tau * tau + t02);
  const R heps = t02 * (R(0.5) * inv);          // eps / 2
  const R dco = tau * inv * R(1.0 / 3.0);       // (1 - eps) / (3 tau)
  const R FnL = (N == 0) ? L.Fx : L.Fy, FnR = (N == 0) ? Q.Fx : Q.Fy;
  Flux3<R> r;
  if constexpr (EIG) {
    const R eps = heps + heps;
    double loL, hiL, loR, hiR;
    m1_signal_speeds(N == 0 ? fxL : fyL, N == 0 ? fyL : fxL, loL, hiL);
    m1_signal_speeds(N == 0 ? fxR : fyR, N == 0 ? fyR : fxR, loR, hiR);
    double sl = fmin(fmin(loL, loR), 0.0), sr = fmax(fmax(hiL, hiR), 0.0);
    R wl, wr, wd;                      // central weights and dissipation factor
    if (sr - sl > 0.0) {
      const double id = 1.0 / (sr - sl);
      wl = (R)(sr * id); wr = (R)(-sl * id); wd = (R)(sl * sr * id);
    } else {
      wl = R(0.5); wr = R(0.5); wd = R(0);
    }
    r.e = eps * (wl * FnL + wr * FnR + wd * (ER - EL)) - dco * dEc;
    r.x = R(2) * (wl * L.hPx + wr * Q.hPx) + eps * wd * (Q.Fx - L.Fx);
    r.y = R(2) * (wl * L.hPy + wr * Q.hPy) + eps * wd * (Q.Fy - L.Fy);
  } else {
    r.e = heps * ((FnL + FnR) - (ER - EL)) - dco * dEc;
    r.x = (L.hPx + Q.hPx) - heps * (Q.Fx - L.Fx);
    r.y = (L.hPy + Q.hPy) - heps * (Q.Fy - L.Fy);
  }
  // upwind advection by the face velocity with the upstream reconstruction
  const bool up = un_c > R(0);
  r.e += un_c * (up ? EL : ER);
  r.x += un_c * (up ? L.Fx : Q.Fx);
  r.y += un_c * (up ? L.Fy : Q.Fy);
  return r;
}

// Emission/absorption (Section 2.1, step 2: BDF1) after the transport step of
// one cell.  E0, fx0, fy0: the state at the start of the step (F = f E);
// dE, dX, dY: the changes of the transport step, so that E* = E0 - dE etc.;
// Es, Xs, Ys: the post-transport state after the causality clamp; kept: the
// clamp left it unchanged; s = c_tilde dt S, x = c_tilde dt kappa_E,
// y = c_tilde dt alpha_F.  Then E** = (E* + s)/(1 + x) and F** = F*/(1 + y).
// Where the clamp kept the state and x < 1 (y < 1), E** is formed as
//   E0 - (dE - s + (E* + s) x/(1 + x))
// (F** as fx0 E0 - (dX + F* y/(1 + y))), so that a step rounds the state once,
// at its own scale: the changes are summed first.  Rounding it after every
// partial update repeats nearly the same error each step in a slowly
// changing field, and in FP32 that error grows linearly over a long run.
template <typename R>
__device__ __forceinline__ void source_update(R E0, R fx0, R fy0, R dE, R dX, R dY, R Es, R Xs,
                                              R Ys, bool kept, R s, R x, R y, R& En, R& Xn,
                                              R& Yn) {
  const R rx = frcp(R(1) + x), ry = frcp(R(1) + y);
  if (kept && x < R(1)) En = E0 - ((dE - s) + (Es + s) * (x * rx));
  else                  En = x < R(1) ? (Es + s) - (Es + s) * (x * rx) : (Es + s) * rx;
  if (kept && y < R(1)) {
    Xn = fx0 * E0 - (dX + Xs * (y * ry));
    Yn = fy0 * E0 - (dY + Ys * (y * ry));
  } else if (y < R(1)) {
    Xn = Xs - Xs * (y * ry);
    Yn = Ys - Ys * (y * ry);
  } else {
    Xn = Xs * ry;
    Yn = Ys * ry;
  }
}

// ---------------------------------------------------------------- K2
// LDS-tiled advection + emission/absorption.  A block owns a tile of
// kTX x kTY cells and walks a run of bins.  Per bin: (1) the tile plus two
// ghost layers of the state (E, f) and the alpha_F ring are staged in LDS,
// (2) every x- and y-face flux of the tile is computed exactly once into LDS,
// (3) each lane updates its cells (two per lane), applies the causality clamp
// and the implicit source, and hands E**, F** to its sink (which stores E**
// and f** = F**/E**, or runs the frequency step on them).
// Blocks are mapped so that the tiles one XCD runs are contiguous in space
// (halo rows shared between neighbouring tiles then hit the same L2).
// 32 x 16 cells: fewer halo cells and faces per cell than 64 x 8 (1.41 vs
// 1.59 staged entries, 2.09 vs 2.14 faces), rows still whole 128-byte lines.
constexpr int kTX = 32, kTY = 16;
constexpr int kRowsPerPass = 256 / kTX;        // tile rows one pass of the block covers
static_assert(kTX * kTY == 512 && 256 % kTX == 0, "a block owns 512 cells, two per lane");
constexpr int kPX = kTX + 4, kPY = kTY + 4;   // padded tile, halo 2
constexpr int kRX = kTX + 2, kRY = kTY + 2;   // opacity ring, halo 1
// LDS row strides: one word more than a row, odd, so that the four rows a
// half-wave of row-wise face runs touches fall in distinct banks.
template <typename R> constexpr int kPad = 1;
template <typename R> constexpr int kPS = kPX + kPad<R>;
template <typename R> constexpr int kRS = kRX + kPad<R>;
constexpr int kNXF = kTY * (kTX + 1);         // x-faces of a tile
constexpr int kNYF = (kTY + 1) * kTX;         // y-faces of a tile

template <typename R>
struct AdvShared {
  R E[kPY][kPS<R>], fx[kPY][kPS<R>], fy[kPY][kPS<R>];  // staged state: E and f = F/E
  int src[kPY * kPX];                          // staging sources (see advect_block)
  R aF[kRY][kRS<R>];                           // alpha_F of the ring, this bin
  R ral[kRX * kRY], racF[kRX * kRY];           // ring: alpha, alpha_cF (fixed over bins)
  R fle[kNXF + kNYF], flx[kNXF + kNYF], fly[kNXF + kNYF];  // face fluxes
  R un[kNXF + kNYF];                           // face-normal velocity / c
  R xidl[kTX + 3], xhp[kTX + 2], xhm[kTX + 2]; // columns x0-1 .. (geometry)
  R yidl[kTY + 3], yhp[kTY + 2], yhm[kTY + 2]; // rows y0-1 ..
};

// Logical block index: XCD x (hardware round-robin b mod 8) gets a
// contiguous range of logical blocks.
__device__ __forceinline__ unsigned xcd_logical_block() {
  const unsigned B = gridDim.x, b = blockIdx.x;
  const unsigned x = b & 7u, slot = b >> 3, q = B >> 3, r = B & 7u;
  return x * q + (x < r ? x : r) + slot;
}

// Source cell of a tile entry (ii, jj) with ghost rules; returns false when
// the entry lies outside the `depth` ghost layers or in a domain corner.
__device__ __forceinline__ bool ghost_source(int ii, int jj, int nx, int ny, const int* bc,
                                             int depth, int& si, int& sj, int& sgx, int& sgy,
                                             bool& vac) {
  si = ii; sj = jj; sgx = 1; sgy = 1; vac = false;
  const bool ox = ii < 0 || ii >= nx, oy = jj < 0 || jj >= ny;
  if (ox && oy) return false;
  if (ox) {
    if (ii < -depth || ii >= nx + depth) return false;
    const int side = ii < 0 ? 0 : 1;
    if (bc[side] != kReflect) { vac = true; return true; }
    si = ii < 0 ? -1 - ii : 2 * nx - 1 - ii;
    sgx = -1;
  } else if (oy) {
    if (jj < -depth || jj >= ny + depth) return false;
    const int side = jj < 0 ? 2 : 3;
    if (bc[side] != kReflect) { vac = true; return true; }
    sj = jj < 0 ? -1 - jj : 2 * ny - 1 - jj;
    sgy = -1;
  }
  return true;
}

constexpr int kRingPerLane = (kRX * kRY + 255) / 256;   // 3
constexpr int kStagePerLane = (kPX * kPY + 255) / 256;  // 3

// Runs of faces: 128 lanes take the kTY x (kTX + 1) x-faces, 128 the
// kTX x (kTY + 1) y-faces, each lane four faces along one line; the last face
// of every line is taken by a second, one-face run (x: wave 0, y: wave 2), so
// no lane of a wave walks a longer run than the others.
constexpr int kRunsX = 128 / kTY;     // runs per tile row
constexpr int kRunsY = 128 / kTX;     // runs per tile column
static_assert(128 % kTY == 0 && 128 % kTX == 0, "runs must tile the faces");
constexpr int kRun = 4;               // faces per run; the last face of a line apart
static_assert(kRunsX * kRun == kTX && kRunsY * kRun == kTY, "runs of four cover a line but its last face");

// Faces per iteration of a run.  Unrolled, a run keeps no register rotation
// between faces and addresses LDS with constant offsets: float fully (four
// waves per SIMD leave it the registers), double by two.  The active-bin and
// substep variants and the fused sink carry more state through the bin loop
// and would spill, so they keep one face per iteration.
template <typename R, bool EXTRA>
constexpr int kFaceUnroll = EXTRA ? 1 : (sizeof(R) == 8 ? 2 : kRun);

// Faces [c0, c1) along line `line` (N = 0: tile row, faces between padded
// columns c+1 and c+2; N = 1: tile column, faces between padded rows c+1 and
// c+2).  MinMod slopes on centroid distances: each cell's slope and each
// difference between neighbours is formed once and carried along the run.
template <typename R, int N, int U, bool EIG = false>
__device__ __forceinline__ void face_run(AdvShared<R>& S, int line, int c0, int c1) {
  auto ld = [&](int p, R& e, R& x, R& y) {
    if (N == 0) { e = S.E[line + 2][p]; x = S.fx[line + 2][p]; y = S.fy[line + 2][p]; }
    else        { e = S.E[p][line + 2]; x = S.fx[p][line + 2]; y = S.fy[p][line + 2]; }
  };
  const R* idl = N == 0 ? S.xidl : S.yidl;
  const R* hp = N == 0 ? S.xhp : S.yhp;
  const R* hm = N == 0 ? S.xhm : S.yhm;
  R e0, x0, y0, e1, x1, y1, e2, x2, y2;
  ld(c0, e0, x0, y0);
  ld(c0 + 1, e1, x1, y1);
  ld(c0 + 2, e2, x2, y2);
  const R i01 = idl[c0];
  R i12 = idl[c0 + 1];
  R dE = (e2 - e1) * i12, dX = (x2 - x1) * i12, dY = (y2 - y1) * i12;
  R sE = minmod((e1 - e0) * i01, dE), sX = minmod((x1 - x0) * i01, dX),
    sY = minmod((y1 - y0) * i01, dY);
  // U faces per iteration (see kFaceUnroll)
#pragma unroll U
  for (int c = c0; c < c1; ++c) {
    R e3, x3, y3;
    ld(c + 3, e3, x3, y3);
    const R i23 = idl[c + 2];
    const R dE3 = (e3 - e2) * i23, dX3 = (x3 - x2) * i23, dY3 = (y3 - y2) * i23;
    const R tE = minmod(dE, dE3), tX = minmod(dX, dX3), tY = minmod(dY, dY3);
    const R hL = hp[c], hR = hm[c + 1];
    R aFL, aFR;
    int f;
    if (N == 0) { aFL = S.aF[line + 1][c]; aFR = S.aF[line + 1][c + 1]; f = line * (kTX + 1) + c; }
    else        { aFL = S.aF[c][line + 1]; aFR = S.aF[c + 1][line + 1]; f = kNXF + c * kTX + line; }
    const Flux3<R> r = face_flux<R, N, EIG>(e1 + sE * hL, x1 + sX * hL, y1 + sY * hL,
                                       e2 + tE * hR, x2 + tX * hR, y2 + tY * hR,
                                       e2 - e1, hL, hR, aFL, aFR, S.un[f]);
    S.fle[f] = r.e; S.flx[f] = r.x; S.fly[f] = r.y;
    e1 = e2; x1 = x2; y1 = y2;
    e2 = e3; x2 = x3; y2 = y3;
    dE = dE3; dX = dX3; dY = dY3;
    sE = tE; sX = tX; sY = tY;
  }
}

// Element c of a bin plane starting at `plane`, addressed as the plane (a
// block-uniform pointer) plus a 32-bit byte offset: a grid holds at most 2^29
// cells, so c * sizeof(R) < 2^32 and the scalar-base + vector-offset form of
// the memory instructions applies.
template <typename R>
__device__ __forceinline__ R* plane_at(R* plane, unsigned c) {
  return (R*)((char*)plane + c * (unsigned)sizeof(R));
}

// Where the post-source state E**, F** of an owned cell goes: to the output
// state (the frequency step runs in its own kernel), or into the frequency
// step of the same block (fused).  A cell is addressed by the offset koff of
// its bin plane and its index c in the plane.
template <typename R>
struct WriteSink {
  static constexpr bool kHeavy = false;     // holds no per-cell state across bins
  __device__ __forceinline__ void init(const GridArgs<R>&, const bool*, const unsigned*,
                                       const int*) {}
  __device__ __forceinline__ void put(const GridArgs<R>& a, int, int, size_t koff, unsigned c,
                                      R h, R E, R X, R Y) {
    (void)h;
    R fxo, fyo;
    reduced_flux<R>(E, X, Y, fxo, fyo);
    __builtin_nontemporal_store(E, plane_at(a.Eo + koff, c));
    __builtin_nontemporal_store(fxo, plane_at(a.fxo + koff, c));
    __builtin_nontemporal_store(fyo, plane_at(a.fyo + koff, c));
  }
  __device__ __forceinline__ void finish(const GridArgs<R>&, const bool*, const unsigned*) {}
};

// Sink of the band step (Section 2.5): stores the state like WriteSink and
// sums the force sum_B kappa_F,B F**_B of its two cells over the bands (in
// double), written once after the last band.  The band loop hands it
// h = kappa_F of the cell and band.  There is no line share: force rows 2
// and 3 are written 0.  Its sums cost the float kernel the registers of the
// unrolled face runs (they would spill); double keeps its two-face unroll.
template <typename R>
struct BandSink {
  static constexpr bool kHeavy = sizeof(R) == 4;
  double fx[2], fy[2];
  __device__ __forceinline__ void init(const GridArgs<R>&, const bool*, const unsigned*,
                                       const int*) {
    fx[0] = fx[1] = fy[0] = fy[1] = 0.0;
  }
  __device__ __forceinline__ void put(const GridArgs<R>& a, int m, int, size_t koff, unsigned c,
                                      R h, R E, R X, R Y) {
    R fxo, fyo;
    reduced_flux<R>(E, X, Y, fxo, fyo);
    __builtin_nontemporal_store(E, plane_at(a.Eo + koff, c));
    __builtin_nontemporal_store(fxo, plane_at(a.fxo + koff, c));
    __builtin_nontemporal_store(fyo, plane_at(a.fyo + koff, c));
    fx[m] += (double)h * (double)X;
    fy[m] += (double)h * (double)Y;
  }
  __device__ __forceinline__ void finish(const GridArgs<R>& a, const bool* own,
                                         const unsigned* cidx) {
    const size_t nc = (size_t)a.nx * a.ny;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      if (!own[m]) continue;
      const size_t c = cidx[m];
      a.force[c] = fx[m];
      a.force[nc + c] = fy[m];
      a.force[2 * nc + c] = 0.0;
      a.force[3 * nc + c] = 0.0;
    }
  }
};

// One tile x run of bins (logical block L of grid a); BK = 0: all bins.
// AB: the grid selects active bins (a.active); a separate instantiation, so
// that grids advecting every bin keep the registers of the plain loop.
// SUB: emission/absorption is left to the frequency kernel (substep rule);
// the sink gets the post-transport state.
// BAND: the grid holds broad bands (Section 2.5): opacities and emission
// come per band and cell from a.kflux, a.kabs, a.jsrc instead of the
// per-cell line data and the class profiles.
// EIG: the interface flux is HLL with the M1 signal speeds (a comparison
// variant; one face per iteration).
template <typename R, int BK, bool AB, bool SUB, class Sink, bool BAND = false, bool EIG = false>
__device__ __forceinline__ void advect_block(const GridArgs<R>& a, const unsigned L,
                                             AdvShared<R>& S, Sink& sink) {
  static_assert(!(BAND && (AB || SUB)), "bands take neither active bins nor substeps");
  const int nx = a.nx, ny = a.ny, nb = a.nb;
  const size_t nc = (size_t)nx * ny;
  const int nbx = (nx + kTX - 1) / kTX, nby = (ny + kTY - 1) / kTY;
  const int bx = (int)(L % (unsigned)nbx);
  const unsigned t1 = L / (unsigned)nbx;
  const int by = (int)(t1 % (unsigned)nby);
  const int bz = BK > 0 ? (int)(t1 / (unsigned)nby) : 0;
  const int x0 = bx * kTX, y0 = by * kTY, k0 = bz * BK;
  const int kend = BK > 0 ? min(k0 + BK, nb) : nb;
  const int tid = threadIdx.x;
  const R inv_c = R(1.0 / kC);

  // ---- once per block: ring opacities (the class or cell of each entry in
  //      registers, its alpha and alpha_cF in LDS), geometry and face
  //      velocities (LDS)
  int rcls[kRingPerLane];
#pragma unroll
  for (int m = 0; m < kRingPerLane; ++m) {
    const int e = tid + 256 * m;
    R al = R(0), acf = R(0);
    rcls[m] = 0;
    if (e < kRX * kRY) {
      const int ri = e % kRX, rj = e / kRX;
      int si, sj, sgx, sgy;
      bool vac;
      if (ghost_source(x0 + ri - 1, y0 + rj - 1, nx, ny, a.bc, 1, si, sj, sgx, sgy, vac) && !vac) {
        const size_t c = (size_t)sj * nx + si;
        if constexpr (BAND) {            // alpha_F = 1 * kappa_F + 0 below
          al = R(1); rcls[m] = (int)c;
        } else {
          al = a.alpha[c]; acf = a.acF[c]; rcls[m] = a.cls[c];
        }
      }
      S.ral[e] = al;
      S.racF[e] = acf;
    }
  }
  for (int e = tid; e < kTX + 3; e += 256) {
    const int gi = x0 - 1 + e;                       // column index, >= -1
    S.xidl[e] = gi <= nx + 1 ? a.xidl[gi + 2] : R(0);
    if (e < kTX + 2) {
      S.xhp[e] = gi <= nx ? a.xhp[gi + 2] : R(0);
      S.xhm[e] = gi <= nx ? a.xhm[gi + 2] : R(0);
    }
  }
  for (int e = tid; e < kTY + 3; e += 256) {
    const int gj = y0 - 1 + e;
    S.yidl[e] = gj <= ny + 1 ? a.yidl[gj + 2] : R(0);
    if (e < kTY + 2) {
      S.yhp[e] = gj <= ny ? a.yhp[gj + 2] : R(0);
      S.yhm[e] = gj <= ny ? a.yhm[gj + 2] : R(0);
    }
  }
  for (int f = tid; f < kNXF + kNYF; f += 256) {
    R u = R(0);
    if (f < kNXF) {
      const int gi = x0 + f % (kTX + 1), gj = y0 + f / (kTX + 1);
      if (gi <= nx && gj < ny) u = a.ufx[(size_t)gj * (nx + 1) + gi] * inv_c;
    } else {
      const int g = f - kNXF;
      const int gi = x0 + g % kTX, gj = y0 + g / kTX;
      if (gi < nx && gj <= ny) u = a.ufy[(size_t)gj * nx + gi] * inv_c;
    }
    S.un[f] = u;
  }

  // ---- per-lane cells: (tx, ty) and (tx, ty + kRowsPerPass)
  const int tx = tid % kTX, ty = tid / kTX;
  bool own[2];
  unsigned cidx[2];                 // cell index in a bin plane (< 2^29)
  int ccls[2];
  R acabs[2], pda[2], em[2], gxx[2], gyy[2], gxy[2], gsum[2], cy[2];
  const int gi = x0 + tx;
  const bool colok = gi < nx;
  const R cxm = colok ? a.cxm[gi] : R(0), cxp = colok ? a.cxp[gi] : R(0);
  const R chp = colok ? a.chp[gi] : R(0);
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const int gj = y0 + ty + kRowsPerPass * m;
    own[m] = colok && gj < ny;
    cidx[m] = own[m] ? (unsigned)(gj * nx + gi) : 0u;
    const size_t c = cidx[m];
    if constexpr (BAND) {
      ccls[m] = 0; acabs[m] = R(0); pda[m] = R(0); em[m] = R(0);
    } else {
      ccls[m] = own[m] ? a.cls[c] : 0;
      acabs[m] = own[m] ? a.acabs[c] : R(0);
      pda[m] = own[m] ? a.pda[c] : R(0);
      em[m] = own[m] ? a.em[c] : R(0);
    }
    gxx[m] = own[m] ? a.grad[c] : R(0);
    gyy[m] = own[m] ? a.grad[nc + c] : R(0);
    gxy[m] = own[m] ? a.grad[2 * nc + c] : R(0);
    gsum[m] = own[m] ? gxx[m] + gyy[m] + a.grad[3 * nc + c] : R(0);   // trace part
    cy[m] = own[m] ? a.cy[gj] : R(0);
  }
  const R ctdt = a.ctdt, ctdt_c = a.ctdt_c;
  sink.init(a, own, cidx, ccls);

  // staging sources, fixed for all bins: the source cell's offset within a
  // bin shifted left by 2, bit 0 / bit 1 set where f_x / f_y change sign
  // (mirror image), -1 for a vacuum ghost.  Each lane reads back only the
  // entries it wrote, so no barrier is needed.
  for (int e = tid; e < kPX * kPY; e += 256) {
    const int pi = e % kPX, pj = e / kPX;
    int si, sj, sgx, sgy;
    bool vac;
    int v = -1;
    if (ghost_source(x0 + pi - 2, y0 + pj - 2, nx, ny, a.bc, 2, si, sj, sgx, sgy, vac) && !vac)
      v = ((sj * nx + si) << 2) | (sgx < 0 ? 1 : 0) | (sgy < 0 ? 2 : 0);
    S.src[e] = v;
  }

  for (int k = k0; k < kend; ++k) {
    const size_t koff = (size_t)k * nc;
    const R* hb = a.hbar + k;
    const R* Ek = a.E + koff;
    const R* Xk = a.fx + koff;
    const R* Yk = a.fy + koff;
    if (AB && a.active != nullptr && a.active[k] == 0) {   // (batches mix grids)
      // a bin not advected this step keeps its state through the transport
      // step (the state is causal already); emission/absorption as below
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        if (!own[m]) continue;
        const unsigned c = cidx[m];
        const R EC = Ek[c], fxc = Xk[c], fyc = Yk[c];
        const int cc = ccls[m];
        const R hC = hb[(size_t)cc * nb];
        if constexpr (SUB) {
          sink.put(a, m, k, koff, c, hC, EC, fxc * EC, fyc * EC);
          continue;
        }
        const R aFC = a.alpha[c] * hC + a.acF[c];
        const R src = em[m] * a.phi[(size_t)cc * nb + k];
        const R kE = acabs[m] + pda[m] * hC;
        R En, Xn, Yn;
        source_update(EC, fxc, fyc, R(0), R(0), R(0), EC, fxc * EC, fyc * EC, true, ctdt * src,
                      ctdt * kE, ctdt * aFC, En, Xn, Yn);
        sink.put(a, m, k, koff, c, hC, En, Xn, Yn);
      }
      continue;
    }
    // (1) stage E and f of the padded tile, and alpha_F of the ring.  Every
    // load of a lane is issued before the first of them is used (a vacuum
    // ghost reads cell 0 of the bin and drops it), so the block waits on
    // memory once per bin rather than once per entry.
    int sv[kStagePerLane];
    R ev[kStagePerLane], xv[kStagePerLane], yv[kStagePerLane], hr[kRingPerLane];
#pragma unroll
    for (int m = 0; m < kStagePerLane; ++m) {
      const int e = tid + 256 * m;
      sv[m] = e < kPX * kPY ? S.src[e] : -1;
      const int q = sv[m] >= 0 ? sv[m] >> 2 : 0;
      ev[m] = Ek[q];
      xv[m] = Xk[q];
      yv[m] = Yk[q];
    }
    R hcell[2], pcell[2], kcell[2];       // profiles of the owned cells for step (3)
    if constexpr (BAND) {
      // kappa_F of the ring, and kappa_F, L/c, kappa_abs of the owned cells
      const R* KF = a.kflux + koff;
#pragma unroll
      for (int m = 0; m < kRingPerLane; ++m) hr[m] = *plane_at(KF, (unsigned)rcls[m]);
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        hcell[m] = *plane_at(KF, cidx[m]);
        pcell[m] = *plane_at(a.jsrc + koff, cidx[m]);
        kcell[m] = *plane_at(a.kabs + koff, cidx[m]);
      }
    } else {
#pragma unroll
      for (int m = 0; m < kRingPerLane; ++m) hr[m] = hb[(size_t)rcls[m] * nb];
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        hcell[m] = hb[(size_t)ccls[m] * nb];
        pcell[m] = a.phi[(size_t)ccls[m] * nb + k];
        kcell[m] = R(0);
      }
    }
#pragma unroll
    for (int m = 0; m < kStagePerLane; ++m) {
      const int e = tid + 256 * m, v = sv[m];
      if (e < kPX * kPY) {
        const int d = e + (e / kPX) * kPad<R>;   // entry (e / kPX, e % kPX) at row stride kPS
        (&S.E[0][0])[d] = v >= 0 ? ev[m] : R(0);
        (&S.fx[0][0])[d] = v < 0 ? R(0) : ((v & 1) ? -xv[m] : xv[m]);
        (&S.fy[0][0])[d] = v < 0 ? R(0) : ((v & 2) ? -yv[m] : yv[m]);
      }
    }
#pragma unroll
    for (int m = 0; m < kRingPerLane; ++m) {
      const int e = tid + 256 * m;
      if (e < kRX * kRY) (&S.aF[0][0])[e + (e / kRX) * kPad<R>] = S.ral[e] * hr[m] + S.racF[e];
    }
    __syncthreads();
    // (2) every face of the tile once, in runs of four consecutive faces
    // along a line: waves 0-1 the x-faces (runs along rows), waves 2-3 the
    // y-faces (runs along columns); then the last face of each line.
    constexpr int FU = kFaceUnroll<R, AB || SUB || EIG || Sink::kHeavy>;
    if (tid < 128) {
      const int r = tid / kRunsX, s = tid % kRunsX;
      face_run<R, 0, FU, EIG>(S, r, s * kRun, s * kRun + kRun);
      if (tid < kTY) face_run<R, 0, 1, EIG>(S, tid, kTX, kTX + 1);   // last face of row tid
    } else {
      // a half-wave takes 32 neighbouring columns at one run position, so
      // its reads and flux writes fall in distinct banks
      const int u = tid - 128, c = u % kTX, s = u / kTX;
      face_run<R, 1, FU, EIG>(S, c, s * kRun, s * kRun + kRun);
      if (u < kTX) face_run<R, 1, 1, EIG>(S, u, kTY, kTY + 1);       // last face of column u
    }
    // The owned cells' staged state and alpha_F, read before the barrier:
    // the update then reads only the fluxes (rewritten after the next bin's
    // first barrier), so the next bin's staging may start while slower waves
    // still update, and no third barrier per bin is needed.
    R Ec[2], fxs[2], fys[2], aFs[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int lj = ty + kRowsPerPass * m;
      Ec[m] = S.E[lj + 2][tx + 2];
      fxs[m] = S.fx[lj + 2][tx + 2];
      fys[m] = S.fy[lj + 2][tx + 2];
      aFs[m] = S.aF[lj + 1][tx + 1];
    }
    __syncthreads();
    // (3) update, causality clamp, implicit source.  Both cells' source
    // coefficients are formed first: a cell-1 value first used after cell 0's
    // stores would make the wave wait for those stores to complete (stores
    // and loads share one counter).
    R srcv[2], kEv[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      srcv[m] = BAND ? pcell[m] : em[m] * pcell[m];
      kEv[m] = BAND ? kcell[m] : acabs[m] + pda[m] * hcell[m];
    }
    asm volatile("" : "+v"(srcv[1]), "+v"(kEv[1]), "+v"(hcell[1]));   // formed here, not later
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      if (!own[m]) continue;
      const int lj = ty + kRowsPerPass * m;
      const R EC = Ec[m], fxc = fxs[m], fyc = fys[m];
      const int w = lj * (kTX + 1) + tx;             // west face; east = w + 1
      const int so = kNXF + lj * kTX + tx;           // south face; north = so + kTX
      // closure of the cell's reduced flux (|f| > 1 scaled back to 1 first);
      // work term D : grad u = iso (gxx + gyy + gpp) + g (fx^2 gxx + fy^2 gyy
      // + fx fy gxy), hoop term from D_phiphi = iso
      R cfx = fxc, cfy = fyc;
      R xx2 = cfx * cfx, yy2 = cfy * cfy;
      if (xx2 + yy2 > R(1)) [[unlikely]] {
        const R sc = frsq(xx2 + yy2);
        cfx *= sc; cfy *= sc;
        xx2 = cfx * cfx; yy2 = cfy * cfy;
      }
      const ClosureParts<R> D = closure_parts(xx2 + yy2);
      const R ddu = D.iso * gsum[m] + D.g * (xx2 * gxx[m] + yy2 * gyy[m] + (cfx * cfy) * gxy[m]);
      // the changes of the transport step (flux divergence, work and hoop
      // terms), summed before they meet the state
      const R dE = (cxp * S.fle[w + 1] - cxm * S.fle[w] + cy[m] * (S.fle[so + kTX] - S.fle[so]))
                   + ctdt_c * ddu * EC;
      const R dX = (cxp * S.flx[w + 1] - cxm * S.flx[w] + cy[m] * (S.flx[so + kTX] - S.flx[so]))
                   - chp * D.iso * EC;
      const R dY = cxp * S.fly[w + 1] - cxm * S.fly[w] + cy[m] * (S.fly[so + kTX] - S.fly[so]);
      R Es = EC - dE;
      R Xs = fxc * EC - dX;
      R Ys = fyc * EC - dY;
      // causality: E >= 0 and |F| <= E
      const bool pos = Es > R(0);
      const R cl = pos ? causal_scale(Es, Xs, Ys) : R(1);
      const bool kept = pos && cl == R(1);          // no clamp: the usual case
      Xs = pos ? Xs * cl : R(0);
      Ys = pos ? Ys * cl : R(0);
      Es = pos ? Es : R(0);
      const R hC = hcell[m];
      const R aFC = aFs[m];
      if constexpr (SUB) {
        sink.put(a, m, k, koff, cidx[m], hC, Es, Xs, Ys);
        continue;
      }
      R En, Xn, Yn;
      source_update(EC, fxc, fyc, dE, dX, dY, Es, Xs, Ys, kept, ctdt * srcv[m], ctdt * kEv[m],
                    ctdt * aFC, En, Xn, Yn);
      sink.put(a, m, k, koff, cidx[m], hC, En, Xn, Yn);
    }
  }
  sink.finish(a, own, cidx);
}

// Float: four waves per SIMD (128 registers), which the fully unrolled face
// runs need; at five (the block count LDS would allow) they spill.
template <typename R>
constexpr int kAdvectWaves = sizeof(R) == 4 ? 4 : 1;

template <typename R, int BK, bool AB, bool SUB, bool EIG = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kAdvectWaves<R>)))
void k_advect_source(GridArgs<R> a) {
  __shared__ AdvShared<R> S;
  WriteSink<R> sink;
  advect_block<R, BK, AB, SUB, WriteSink<R>, false, EIG>(a, xcd_logical_block(), S, sink);
}

// The step of a grid of broad bands (Section 2.5): a block per tile walks
// all bands, so its sink sums the force over them; no frequency step.
template <typename R>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kAdvectWaves<R>)))
void k_band_step(GridArgs<R> a) {
  __shared__ AdvShared<R> S;
  BandSink<R> sink;
  advect_block<R, 0, false, false, BandSink<R>, true>(a, xcd_logical_block(), S, sink);
}

// Batched advection: one launch covers the work items (grid, tile x run of
// bins) of every grid of a batch.  A block takes the item of its XCD-ordered
// index (and, when a batch has more items than the launch has blocks, every
// grid-size stride after it), so that the blocks of one XCD work on one
// contiguous range of tiles and share its halo lines in their L2.  The host
// launches a block per item: the hardware then balances the blocks over the
// CUs (a persistent grid of CUs x occupancy blocks was 9 % slower: its
// blocks stay in step through the per-item set-up).  off[g] is the
// first work item of grid g (off[n] = total); args holds both ping-pong
// directions, [2][n]; grid g uses direction par[g] ^ sp.
template <typename R, int BK, bool AB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kAdvectWaves<R>)))
void k_advect_batched(const GridArgs<R>* __restrict__ args,
                                                        const int* __restrict__ par, int n,
                                                        int sp, const int* __restrict__ off) {
  __shared__ AdvShared<R> S;
  const int total = off[n];
  for (int w = (int)xcd_logical_block(); w < total; w += gridDim.x) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (off[mid] <= w) lo = mid; else hi = mid;
    }
    const GridArgs<R> a = global_args(args[((par[lo] ^ sp) & 1) * n + lo]);
    WriteSink<R> sink;
    advect_block<R, BK, AB, false>(a, (unsigned)(w - off[lo]), S, sink);
  }
}

// ---------------------------------------------------------------- K3
// E1(z) = (e^z - 1)/z by its Taylor series, for |z| < 1/2.
template <typename T>
__device__ __forceinline__ T e1_series(T z) {
  constexpr int n = sizeof(T) == 8 ? 16 : 9;     // last term < 2e-18 / 2e-9
  T r = T(1);
#pragma unroll
  for (int j = n; j >= 1; --j) r = T(1) + z * r * (T(1) / T(j + 1));   // 1/(j+1) folds
  return r;
}

// e^x.  Float: the hardware's 2^t with t = x log2(e) carried to about 2^-40
// (head product, its rounding error by FMA, and the tail of log2(e)), so the
// result keeps about 1 ulp; x = 0 gives exactly 1.  Arguments below -150
// give 0.  Double: the library exp.
__device__ __forceinline__ double fexp(double x) { return exp(x); }
__device__ __forceinline__ float fexp(float x) {
  x = x > -150.0f ? x : -150.0f;
  const float L = 1.44269502162933349609375f;        // log2(e) rounded to float
  const float Llo = 1.92596298909109e-8f;             // log2(e) - L
  const float t = x * L;
  const float err = __builtin_fmaf(x, L, -t) + x * Llo;
  return __builtin_amdgcn_exp2f(t) * (1.0f + err * 0.693147180559945309f);
}

// Exponential-scheme interface between bins l < r (frequency flux
// F = gr J_r - gl J_l):  gl = e^{A}/den, gr = e^{B}/den with A = -P_l =
// -Cl ql, B = P_r = Cr qr, den = ql E1(A) + qr E1(B), ql = dl/Kl, qr = dr/Kr,
// E1(z) = (e^z - 1)/z.  Numerator and denominator are scaled by e^{-m},
// m = max(A, B, 0) (an exact rewrite), so every exponential is <= 1 and
// e^{-m} E1(z) <= 2: nothing overflows at any Peclet number.  E1 is taken
// from its series for |z| < 1/2, else from (e^{z-m} - e^{-m})/z.  Of the
// three exponents A - m, B - m and -m the one that attains the maximum is
// exactly 0, so two exponentials give all three factors.
template <typename T>
__device__ __forceinline__ void interface_rates(T ql, T Cl, T qr, T Cr, T& gl, T& gr) {
  // No contraction here: A - m must be exactly 0 on the dominant side.  A
  // fused multiply-subtract of -Cl*ql - m would leave the rounding error of
  // A (large when |A| ~ 1e10) in the exponent.
#pragma clang fp contract(off)
  const T A = -Cl * ql, B = Cr * qr;
  const bool Alo = A < B;
  const T lo = Alo ? A : B, hi = Alo ? B : A;
  const bool pos = hi >= T(0);           // m = hi, else m = 0
  const T e1 = fexp(pos ? lo - hi : lo);  // e^{lo - m}
  const T e2 = fexp(pos ? -hi : hi);      // e^{-m}, else e^{hi - m}
  const T ehi = pos ? T(1) : e2, em = pos ? e2 : T(1);
  const T eAm = Alo ? e1 : ehi, eBm = Alo ? ehi : e1;
  // |A|, |B| >= 1/2 on the division branches; den is positive
  const T sA = fabs(A) < T(0.5) ? em * e1_series(A) : (eAm - em) * frcp(A);
  const T sB = fabs(B) < T(0.5) ? em * e1_series(B) : (eBm - em) * frcp(B);
  const T den = ql * sA + qr * sB;
  const T iden = den >= recip_floor<T>() ? frcp(den) : T(1) / den;
  gl = eAm * iden;
  gr = eBm * iden;
}

// Coefficients of bin k of one cell (Appendix A): q = (dnu_k/2)/K_k, with
// K_k = (dnu_D^2/2) alpha <H>_k (q = 0 flags a bin without line opacity), and
// C_k = K_k R_k + (nu_k/c) D_k : grad u, D from the post-source reduced flux.
template <typename R, typename T>
struct FreqCell {
  T dd, hkT, gxx, gyy, gxy, gpp;
  bool recoil, doppler;
  __device__ __forceinline__ void coeffs(const GridArgs<R>& a, int k, R h, R fx, R fy, T& q,
                                         T& C) const {
    coeffs_of(a.two_nu[k], a.nu_c[k], a.dnu[k], h, fx, fy, q, C);
  }
  // The same with bin k's table entries (2/nu_k, nu_k/c, dnu_k) passed in: a
  // caller whose k is uniform loads them before any divergent branch, so
  // they stay scalar loads that no vector-memory wait depends on.
  __device__ __forceinline__ void coeffs_of(double two_nu, double nu_c, double dnu, R h, R fx,
                                            R fy, T& q, T& C) const {
    const T K = dd * (T)h;
    T Cv = T(0);
    if (recoil) Cv += K * (hkT - (T)two_nu);
    if (doppler) {
      const Eddington<T> D = closure_reduced<T>((T)fx, (T)fy);
      Cv += (T)nu_c * (D.xx * gxx + D.yy * gyy + D.xy * gxy + D.pp * gpp);
    }
    C = Cv;
    const T hdnu = (T)(0.5 * dnu);
    q = K >= recip_floor<T>() ? hdnu * frcp(K) : (K > T(0) ? hdnu / K : T(0));
  }
};

// One row of the forward elimination (double).  With r1 = s_{k-1}/p_{k-1} and
// r2 = a_{k-1} z_{k-1}:  s_k = 1 + b_k r1,  d_k = y_k + r2,  p_k = s_k + a_k,
// z_k = d_k/p_k,  w_k = b_{k+1}/p_k.
struct FreqRow {
  double r1 = 0.0, r2 = 0.0;
  double b = 0.0;                  // rate of bin k toward k-1 (zero at the lower end)
  template <typename R>
  __device__ __forceinline__ void eliminate(int k, double y, double a_k, double b_next,
                                            ZW<R>* __restrict__ out) {
    const double s = (k == 0) ? 1.0 : 1.0 + b * r1;
    const double d = (k == 0) ? y : y + r2;
    const double ip = frcp(s + a_k);       // s + a_k >= 1
    const double z = d * ip;
    __builtin_nontemporal_store((R)z, &out->z);
    __builtin_nontemporal_store((R)(b_next * ip), &out->w);
    r1 = s * ip;
    r2 = a_k * z;
    b = b_next;
  }
};

// Forward elimination over the bins of one cell: writes z_k = d_k/p_k and
// w_k = b_{k+1}/p_k, accumulates the force.  The state is only read here
// and the scratch only written.  With double storage the loads of a bin are
// issued one bin ahead of their use (the latency dominates there); with
// float storage they are issued just in time, which keeps the register count
// at full occupancy.
template <typename R, typename T>
__device__ __forceinline__ void freq_forward(const GridArgs<R>& a, const FreqCell<R, T>& fc,
                                             size_t c, size_t nc, const R* __restrict__ Ein,
                                             const R* __restrict__ Xin,
                                             const R* __restrict__ Yin, const R* __restrict__ hb,
                                             ZW<R>* __restrict__ zw, T al,
                                             double acF, double* f4) {
  const int nb = a.nb;
  const double ctdt = (double)a.ctdt;
  double fx = 0.0, fy = 0.0, gx = 0.0, gy = 0.0;
  auto force = [&](int k, R h, R e, R rx, R ry) {
    // force density: sum_k dnu_k alpha_F,k F**_k (and the line part)
    const double dn = a.dnu[k];
    const double aH = (double)al * (double)h;
    const double aF = aH + acF;
    const double X = (double)rx * (double)e, Y = (double)ry * (double)e;
    fx += dn * aF * X;
    fy += dn * aF * Y;
    gx += dn * aH * X;
    gy += dn * aH * Y;
  };
  constexpr bool kAhead = sizeof(R) == 8;
  R e0 = Ein[c], x0 = Xin[c], y0 = Yin[c], h0 = hb[0];
  R e1 = R(0), x1 = R(0), y1 = R(0), h1 = R(0);
  if (kAhead && nb > 1) { e1 = Ein[nc + c]; x1 = Xin[nc + c]; y1 = Yin[nc + c]; h1 = hb[1]; }
  T qc, Cc;
  fc.coeffs(a, 0, h0, x0, y0, qc, Cc);
  force(0, h0, e0, x0, y0);
  FreqRow row;
  for (int k = 0; k < nb; ++k) {
    R e2 = R(0), x2 = R(0), y2 = R(0), h2 = R(0);
    if constexpr (kAhead) {
      if (k + 2 < nb) {
        const size_t i2 = (size_t)(k + 2) * nc + c;
        e2 = Ein[i2]; x2 = Xin[i2]; y2 = Yin[i2]; h2 = hb[k + 2];
      }
    } else if (k + 1 < nb) {
      const size_t i1 = (size_t)(k + 1) * nc + c;
      e1 = Ein[i1]; x1 = Xin[i1]; y1 = Yin[i1]; h1 = hb[k + 1];
    }
    double a_k = 0.0, b_next = 0.0;
    if (k + 1 < nb) {
      const double tn = a.two_nu[k + 1], vc = a.nu_c[k + 1], dn = a.dnu[k + 1];
      T qn, Cn;
      fc.coeffs_of(tn, vc, dn, h1, x1, y1, qn, Cn);
      force(k + 1, h1, e1, x1, y1);
      T gl, gr;
      if (qc > T(0) && qn > T(0)) {
        interface_rates<T>(qc, Cc, qn, Cn, gl, gr);
      } else {
        gl = Cc < T(0) ? -Cc : T(0);       // K -> 0: first-order upwind
        gr = Cn > T(0) ? Cn : T(0);
      }
      a_k = ctdt * (double)gl * a.inv_dnu[k];
      b_next = ctdt * (double)gr * a.inv_dnu[k + 1];
      qc = qn;
      Cc = Cn;
    }
    row.eliminate<R>(k, a.dnu[k] * (double)e0, a_k, b_next, &zw[(size_t)k * nc + c]);
    e0 = e1;
    if constexpr (kAhead) { e1 = e2; x1 = x2; y1 = y2; h1 = h2; }
  }
  f4[0] = fx; f4[1] = fy; f4[2] = gx; f4[3] = gy;
}

// Back substitution y_k = z_k + w_k y_{k+1}, E^{n+1} = y/dnu, in place.  The
// H rescale F^{n+1} = (F**/E**) E^{n+1} keeps the stored reduced flux.
template <typename R>
__device__ __forceinline__ void freq_backward(const GridArgs<R>& a, size_t c, size_t nc,
                                              R* __restrict__ Eio,
                                              const ZW<R>* __restrict__ zw) {
  double y = 0.0;
  int k = a.nb - 1;
  // the loads of G bins at a time, then their G dependent steps: one load in
  // flight per wave would leave this memory-bound sweep waiting on latency
  constexpr int G = 8;
  for (; k >= G - 1; k -= G) {
    ZW<R> v[G];
#pragma unroll
    for (int j = 0; j < G; ++j) {
      const size_t idx = (size_t)(k - j) * nc + c;
      v[j].z = __builtin_nontemporal_load(&zw[idx].z);
      v[j].w = __builtin_nontemporal_load(&zw[idx].w);
    }
#pragma unroll
    for (int j = 0; j < G; ++j) {
      y = (double)v[j].z + (double)v[j].w * y;
      __builtin_nontemporal_store((R)(y * a.inv_dnu[k - j]), &Eio[(size_t)(k - j) * nc + c]);
    }
  }
  for (; k >= 0; --k) {
    const size_t idx = (size_t)k * nc + c;
    ZW<R> v;
    v.z = __builtin_nontemporal_load(&zw[idx].z);
    v.w = __builtin_nontemporal_load(&zw[idx].w);
    y = (double)v.z + (double)v.w * y;
    __builtin_nontemporal_store((R)(y * a.inv_dnu[k]), &Eio[idx]);
  }
}

// Frequency step and force of one cell.  R: storage type; T: arithmetic of
// the exponential-scheme coefficients.  The elimination always runs in double.
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
// Per-cell constants of the frequency step of cell c of class cl.
template <typename R, typename T>
__device__ __forceinline__ FreqCell<R, T> freq_cell_consts(const GridArgs<R>& a, size_t c,
                                                           size_t nc, int cl, T al) {
  FreqCell<R, T> fc;
  fc.gxx = (T)a.grad[c];
  fc.gyy = (T)a.grad[nc + c];
  fc.gxy = (T)a.grad[2 * nc + c];
  fc.gpp = (T)a.grad[3 * nc + c];
  fc.dd = (T)a.dD2h[cl] * al;           // 0.5 dnu_D^2 alpha
  fc.hkT = (T)a.hkT[cl];
  fc.recoil = a.recoil != 0;
  fc.doppler = a.doppler != 0 &&
      ((fc.gxx != T(0)) || (fc.gyy != T(0)) || (fc.gxy != T(0)) || (fc.gpp != T(0)));
  return fc;
}

template <typename R, typename T>
__device__ void freq_cell(const GridArgs<R>& a, size_t c) {
  const size_t nc = (size_t)a.nx * a.ny;
  const int cl = a.cls[c];
  const T al = (T)a.alpha[c];
  const FreqCell<R, T> fc = freq_cell_consts<R, T>(a, c, nc, cl, al);
  double f4[4];
  freq_forward<R, T>(a, fc, c, nc, a.Eo, a.fxo, a.fyo, a.hbar + (size_t)cl * a.nb, a.zw,
                     al, (double)a.acF[c], f4);
  freq_backward<R>(a, c, nc, a.Eo, a.zw);
  a.force[c] = f4[0];
  a.force[nc + c] = f4[1];
  a.force[2 * nc + c] = f4[2];
  a.force[3 * nc + c] = f4[3];
}

// Pass 0 steps every cell of a double grid and the non-island cells of a
// float grid (coefficients in float); pass 1 the island cells of a float grid
// (coefficients in double).  Separate kernels, so the rare double-coefficient
// code does not set the register budget of the common one.
template <typename R, int P>
__device__ __forceinline__ void freq_dispatch(const GridArgs<R>& a, size_t c) {
  if constexpr (sizeof(R) == 8) {
    freq_cell<R, double>(a, c);
  } else if constexpr (P == 0) {
    if (!a.island[c]) freq_cell<R, float>(a, c);
  } else {
    if (a.island[c]) freq_cell<R, double>(a, c);
  }
}

// The float pass fits 64 registers: eight waves per SIMD hide its latency.
template <typename R, int P>
constexpr int kFreqWaves = (sizeof(R) == 4 && P == 0) ? 8 : 1;

template <typename R, int P>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kFreqWaves<R, P>)))
void k_freq(GridArgs<R> a) {
  const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (size_t)a.nx * a.ny) return;
  freq_dispatch<R, P>(a, c);
}

// ------------------------------------------- K3 for small grids
// A grid of few cells leaves most of the GPU idle in k_freq, and each lane's
// sweep over the bins is bound by the latency of its ~150 dependent
// instructions per bin, mostly the exponential-scheme coefficients.  Small
// grids therefore take the step in two launches with the same arithmetic:
// k_freq_rates gives every (cell, interface k+1/2) a lane for the rates
// gl, gr of Appendix A (stored in the elimination scratch slot k), then
// k_freq_solve runs the light sequential part per cell (elimination in
// double, force sum, back substitution), with its loads kSolveAhead bins
// ahead.  Non-island cells (island cells of a float grid keep k_freq<R, 1>).
// The rates launch evaluates every bin's coefficients twice at full-chip
// cost, so its time grows with the cell count while k_freq's latency-bound
// time does not, below a round of blocks.  Measured (uniform clouds, 194
// bins, one grid): float 64^2 259 -> 118 us, 128^2 295 -> 174 us, 256^2
// 307 -> 284 us, but a batch of 8 x 128^2 loses (0.64 -> 0.74 ms per step);
// double 128^2 353 -> 233 us, 256^2 383 -> 442 us.  Hence the cut-overs
// below (cells of the launch).
constexpr int kSolveAhead = 4;
template <typename R>
constexpr size_t kTwoPhaseCells = sizeof(R) == 4 ? size_t(1) << 16 : size_t(1) << 15;

// Rates of interface k+1/2 of cell c for t = k ncell + c < (N_nu - 1) ncell.
template <typename R>
__device__ __forceinline__ void freq_rates_at(const GridArgs<R>& a, size_t t) {
  using T = R;                      // float grids: float coefficients (non-island cells)
  const size_t nc = (size_t)a.nx * a.ny;
  const int k = (int)(t / nc);
  const size_t c = t - (size_t)k * nc;
  if (sizeof(R) == 4 && a.island[c]) return;
  const int cl = a.cls[c];
  const T al = (T)a.alpha[c];
  const FreqCell<R, T> fc = freq_cell_consts<R, T>(a, c, nc, cl, al);
  const R* hb = a.hbar + (size_t)cl * a.nb;
  T q0, C0, q1, C1;
  fc.coeffs(a, k, hb[k], a.fxo[t], a.fyo[t], q0, C0);
  fc.coeffs(a, k + 1, hb[k + 1], a.fxo[t + nc], a.fyo[t + nc], q1, C1);
  T gl, gr;
  if (q0 > T(0) && q1 > T(0)) {
    interface_rates<T>(q0, C0, q1, C1, gl, gr);
  } else {
    gl = C0 < T(0) ? -C0 : T(0);       // K -> 0: first-order upwind
    gr = C1 > T(0) ? C1 : T(0);
  }
  ZW<R> v;
  v.z = gl;
  v.w = gr;
  a.zw[t] = v;
}

// Elimination, force and back substitution of cell c after freq_rates_at.
template <typename R>
__device__ __forceinline__ void freq_solve_cell(const GridArgs<R>& a, size_t c) {
  using T = R;
  const size_t nc = (size_t)a.nx * a.ny;
  if (sizeof(R) == 4 && a.island[c]) return;
  const int nb = a.nb;
  const int cl = a.cls[c];
  const T al = (T)a.alpha[c];
  const double acF = (double)a.acF[c];
  const R* hb = a.hbar + (size_t)cl * nb;
  const double ctdt = (double)a.ctdt;
  double fx = 0.0, fy = 0.0, gx = 0.0, gy = 0.0;
  // ring: slot j holds bin k + j (state, profile, rates of interface k+j+1/2)
  R re[kSolveAhead], rx[kSolveAhead], ry[kSolveAhead], rh[kSolveAhead];
  ZW<R> rr[kSolveAhead];
  auto load = [&](int kb, R& e, R& x, R& y, R& h, ZW<R>& r) {
    e = x = y = h = R(0);
    r.z = r.w = R(0);
    if (kb < nb) {
      const size_t i = (size_t)kb * nc + c;
      e = a.Eo[i]; x = a.fxo[i]; y = a.fyo[i]; h = hb[kb];
      if (kb + 1 < nb) r = a.zw[i];
    }
  };
#pragma unroll
  for (int j = 0; j < kSolveAhead; ++j) load(j, re[j], rx[j], ry[j], rh[j], rr[j]);
  FreqRow row;
  for (int k = 0; k < nb; ++k) {
    const R e = re[0], x = rx[0], y = ry[0], h = rh[0];
    const ZW<R> r = rr[0];
#pragma unroll
    for (int j = 0; j + 1 < kSolveAhead; ++j) {
      re[j] = re[j + 1]; rx[j] = rx[j + 1]; ry[j] = ry[j + 1]; rh[j] = rh[j + 1];
      rr[j] = rr[j + 1];
    }
    load(k + kSolveAhead, re[kSolveAhead - 1], rx[kSolveAhead - 1], ry[kSolveAhead - 1],
         rh[kSolveAhead - 1], rr[kSolveAhead - 1]);
    {
      // force density, in bin order as in freq_forward
      const double dn = a.dnu[k];
      const double aH = (double)al * (double)h;
      const double aF = aH + acF;
      const double X = (double)x * (double)e, Y = (double)y * (double)e;
      fx += dn * aF * X;
      fy += dn * aF * Y;
      gx += dn * aH * X;
      gy += dn * aH * Y;
    }
    double a_k = 0.0, b_next = 0.0;
    if (k + 1 < nb) {
      a_k = ctdt * (double)r.z * a.inv_dnu[k];
      b_next = ctdt * (double)r.w * a.inv_dnu[k + 1];
    }
    row.eliminate<R>(k, a.dnu[k] * (double)e, a_k, b_next, &a.zw[(size_t)k * nc + c]);
  }
  freq_backward<R>(a, c, nc, a.Eo, a.zw);
  a.force[c] = fx;
  a.force[nc + c] = fy;
  a.force[2 * nc + c] = gx;
  a.force[3 * nc + c] = gy;
}

template <typename R>
__global__ __launch_bounds__(256) void k_freq_rates(GridArgs<R> a) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < (size_t)(a.nb - 1) * a.nx * a.ny) freq_rates_at<R>(a, t);
}

template <typename R>
__global__ __launch_bounds__(256) void k_freq_solve(GridArgs<R> a) {
  const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < (size_t)a.nx * a.ny) freq_solve_cell<R>(a, c);
}

// ------------------------------------------- K3 with the substep rule
// Section 2.1, step 2, with substeps: the advection kernel leaves the
// emission/absorption to this kernel, which runs it per cell over all bins.
// A substep of a fraction h of the step maps E -> (E + ctdt h S)/(1 + ctdt h kE)
// and F -> F/(1 + ctdt h aF) in every bin (S = em phi_k, kE = acabs + pda
// h_k, aF = alpha h_k + acF); it is accepted when the energy density
// e = sum_k dnu_k E_k changes by less than 0.1 (e + e_floor), else halved and
// redone; after an accepted substep the next one tries twice its length,
// clipped to the time left.  A substep of 2^-60 of the step, or the 4096th
// attempt, is accepted as it is.  Sums, decisions and updates in double.
template <typename R>
struct SourceCell {
  const R* hb;      // the cell's class row of hbar
  const R* ph;      // and of phi
  double em, acabs, pda, al, acF;
  __device__ __forceinline__ void at(int k, double& S, double& kE, double& aH, double& aF) const {
    const double h = (double)hb[k];
    S = em * (double)ph[k];
    kE = acabs + pda * h;
    aH = al * h;
    aF = aH + acF;
  }
};

constexpr int kSubMaxAttempts = 4096;

// Whether the whole step passes the rule (then nothing is written and the
// forward sweep applies the single substep); otherwise the substeps are
// applied to the stored state (E and f, in place) and f4 gets the
// step-averaged force sum_s h_s sum_k dnu_k aF F_k(after s) and its line part.
template <typename R>
__device__ bool source_substeps(const GridArgs<R>& a, size_t c, size_t nc,
                                const SourceCell<R>& sc, double* f4) {
  const int nb = a.nb;
  const double ctdt = (double)a.ctdt, efl = a.e_floor;
  R* __restrict__ Ek = a.Eo;
  R* __restrict__ Xk = a.fxo;
  R* __restrict__ Yk = a.fyo;
  auto energies = [&](double ch, double& e0, double& e1) {
    e0 = 0.0; e1 = 0.0;
    for (int k = 0; k < nb; ++k) {
      double S, kE, aH, aF;
      sc.at(k, S, kE, aH, aF);
      const double E = (double)Ek[(size_t)k * nc + c];
      e0 += a.dnu[k] * E;
      e1 += a.dnu[k] * ((E + ch * S) / (1.0 + ch * kE));
    }
  };
  double e0, e1;
  energies(ctdt, e0, e1);
  f4[0] = f4[1] = f4[2] = f4[3] = 0.0;
  if (fabs(e1 - e0) < 0.1 * (e0 + efl)) return true;
  double done = 0.0, h = 0.5;
  for (int attempt = 2; done < 1.0; ++attempt) {
    if (h > 1.0 - done) h = 1.0 - done;
    const double ch = ctdt * h;
    energies(ch, e0, e1);
    const bool ok = fabs(e1 - e0) < 0.1 * (e0 + efl) || h <= 0x1p-60 ||
                    attempt >= kSubMaxAttempts;
    if (!ok) { h *= 0.5; continue; }
    for (int k = 0; k < nb; ++k) {
      double S, kE, aH, aF;
      sc.at(k, S, kE, aH, aF);
      const size_t i = (size_t)k * nc + c;
      const double E = (double)Ek[i];
      const double E1 = (E + ch * S) / (1.0 + ch * kE);
      const double d = 1.0 / (1.0 + ch * aF);
      const double Fx = (double)Xk[i] * E * d, Fy = (double)Yk[i] * E * d;
      // substep force sum_k dnu_k (F. - F..)/(c dt_sub) = sum_k dnu_k aF F..,
      // weighted by the substep's share h of the step
      const double w = a.dnu[k] * h;
      f4[0] += w * aF * Fx; f4[1] += w * aF * Fy;
      f4[2] += w * aH * Fx; f4[3] += w * aH * Fy;
      Ek[i] = (R)E1;
      Xk[i] = E1 > 0.0 ? (R)(Fx / E1) : R(0);
      Yk[i] = E1 > 0.0 ? (R)(Fy / E1) : R(0);
    }
    done += h;
    h *= 2.0;
  }
  return false;
}

// Forward elimination of one cell reading the post-transport state (full:
// the single substep is applied to each bin on the way, the reduced flux
// after it stored, and the force accumulated) or the post-source state left
// by the substeps.  The steps of freq_forward, a bin at a time.
template <typename R, typename T>
__device__ void freq_forward_sub(const GridArgs<R>& a, const FreqCell<R, T>& fc,
                                 const SourceCell<R>& sc, size_t c, size_t nc, bool full,
                                 double* f4) {
  const int nb = a.nb;
  const double ctdt = (double)a.ctdt;
  T qp = T(0), Cp = T(0);
  R ep = R(0);
  FreqRow row;
  for (int k = 0; k < nb; ++k) {
    const size_t i = (size_t)k * nc + c;
    R e = a.Eo[i], x = a.fxo[i], y = a.fyo[i];
    const R h = sc.hb[k];
    if (full) {
      double S, kE, aH, aF;
      sc.at(k, S, kE, aH, aF);
      const double E = (double)e;
      const double E1 = (E + ctdt * S) / (1.0 + ctdt * kE);
      const double d = 1.0 / (1.0 + ctdt * aF);
      const double Fx = (double)x * E * d, Fy = (double)y * E * d;
      e = (R)E1;
      x = E1 > 0.0 ? (R)(Fx / E1) : R(0);
      y = E1 > 0.0 ? (R)(Fy / E1) : R(0);
      a.fxo[i] = x;
      a.fyo[i] = y;
      const double X = (double)x * (double)e, Y = (double)y * (double)e;
      const double aHr = sc.al * (double)h, aFr = aHr + sc.acF;
      f4[0] += a.dnu[k] * aFr * X; f4[1] += a.dnu[k] * aFr * Y;
      f4[2] += a.dnu[k] * aHr * X; f4[3] += a.dnu[k] * aHr * Y;
    }
    T qk, Ck;
    fc.coeffs(a, k, h, x, y, qk, Ck);
    if (k > 0) {
      T gl, gr;
      if (qp > T(0) && qk > T(0)) {
        interface_rates<T>(qp, Cp, qk, Ck, gl, gr);
      } else {
        gl = Cp < T(0) ? -Cp : T(0);
        gr = Ck > T(0) ? Ck : T(0);
      }
      const double a_k = ctdt * (double)gl * a.inv_dnu[k - 1];
      const double b_next = ctdt * (double)gr * a.inv_dnu[k];
      row.eliminate<R>(k - 1, a.dnu[k - 1] * (double)ep, a_k, b_next,
                       &a.zw[(size_t)(k - 1) * nc + c]);
    }
    qp = qk;
    Cp = Ck;
    ep = e;
  }
  row.eliminate<R>(nb - 1, a.dnu[nb - 1] * (double)ep, 0.0, 0.0,
                   &a.zw[(size_t)(nb - 1) * nc + c]);
}

template <typename R, typename T>
__device__ void freq_cell_sub(const GridArgs<R>& a, size_t c) {
  const size_t nc = (size_t)a.nx * a.ny;
  const int cl = a.cls[c];
  FreqCell<R, T> fc;
  const T al = (T)a.alpha[c];
  fc.gxx = (T)a.grad[c];
  fc.gyy = (T)a.grad[nc + c];
  fc.gxy = (T)a.grad[2 * nc + c];
  fc.gpp = (T)a.grad[3 * nc + c];
  fc.dd = (T)a.dD2h[cl] * al;
  fc.hkT = (T)a.hkT[cl];
  fc.recoil = a.recoil != 0;
  fc.doppler = a.doppler != 0 &&
      ((fc.gxx != T(0)) || (fc.gyy != T(0)) || (fc.gxy != T(0)) || (fc.gpp != T(0)));
  SourceCell<R> sc;
  sc.hb = a.hbar + (size_t)cl * a.nb;
  sc.ph = a.phi + (size_t)cl * a.nb;
  sc.em = (double)a.em[c];
  sc.acabs = (double)a.acabs[c];
  sc.pda = (double)a.pda[c];
  sc.al = (double)a.alpha[c];
  sc.acF = (double)a.acF[c];
  double f4[4];
  const bool full = source_substeps<R>(a, c, nc, sc, f4);
  freq_forward_sub<R, T>(a, fc, sc, c, nc, full, f4);
  freq_backward<R>(a, c, nc, a.Eo, a.zw);
  a.force[c] = f4[0];
  a.force[nc + c] = f4[1];
  a.force[2 * nc + c] = f4[2];
  a.force[3 * nc + c] = f4[3];
}

// Pass P as in k_freq (float: island cells in their own pass).
template <typename R, int P>
__global__ __launch_bounds__(256) void k_freq_sub(GridArgs<R> a) {
  const size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (size_t)a.nx * a.ny) return;
  if constexpr (sizeof(R) == 8) {
    freq_cell_sub<R, double>(a, c);
  } else if constexpr (P == 0) {
    if (!a.island[c]) freq_cell_sub<R, float>(a, c);
  } else {
    if (a.island[c]) freq_cell_sub<R, double>(a, c);
  }
}

// Batched frequency step: work item = 256 cells of one grid (a block per
// item, as for the advection).
template <typename R, int P>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kFreqWaves<R, P>)))
void k_freq_batched(const GridArgs<R>* __restrict__ args,
                                                      const int* __restrict__ par, int n, int sp,
                                                      const int* __restrict__ off) {
  const int total = off[n];
  for (int w = blockIdx.x; w < total; w += gridDim.x) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (off[mid] <= w) lo = mid; else hi = mid;
    }
    const GridArgs<R> a = global_args(args[((par[lo] ^ sp) & 1) * n + lo]);
    const size_t c = (size_t)(w - off[lo]) * 256 + threadIdx.x;
    if (c < (size_t)a.nx * a.ny) freq_dispatch<R, P>(a, c);
  }
}

// The two launches of the small-grid frequency step for a batch: work item
// = 256 interfaces (rates; off = offr) or 256 cells (solve; off = offf).
template <typename R>
__device__ __forceinline__ int batch_member(const int* __restrict__ off, int n, int w) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= w) lo = mid; else hi = mid;
  }
  return lo;
}

template <typename R>
__global__ __launch_bounds__(256) void k_freq_rates_batched(const GridArgs<R>* __restrict__ args,
                                                            const int* __restrict__ par, int n,
                                                            int sp, const int* __restrict__ off) {
  const int total = off[n];
  for (int w = blockIdx.x; w < total; w += gridDim.x) {
    const int g = batch_member<R>(off, n, w);
    const GridArgs<R> a = global_args(args[((par[g] ^ sp) & 1) * n + g]);
    const size_t t = (size_t)(w - off[g]) * 256 + threadIdx.x;
    if (t < (size_t)(a.nb - 1) * a.nx * a.ny) freq_rates_at<R>(a, t);
  }
}

template <typename R>
__global__ __launch_bounds__(256) void k_freq_solve_batched(const GridArgs<R>* __restrict__ args,
                                                            const int* __restrict__ par, int n,
                                                            int sp, const int* __restrict__ off) {
  const int total = off[n];
  for (int w = blockIdx.x; w < total; w += gridDim.x) {
    const int g = batch_member<R>(off, n, w);
    const GridArgs<R> a = global_args(args[((par[g] ^ sp) & 1) * n + g]);
    const size_t c = (size_t)(w - off[g]) * 256 + threadIdx.x;
    if (c < (size_t)a.nx * a.ny) freq_solve_cell<R>(a, c);
  }
}

// ------------------------------------------------------------ fused K2+K3
// Float storage without island cells: the frequency step runs inside the
// advection block.  The block walks all bins of its tile; each owned cell's
// post-source state E**, F** of bin k feeds that cell's forward elimination
// at once (the rates of interface k-1|k need both bins, so row k-1 is
// eliminated when bin k arrives), and after the last bin the block
// back-substitutes its cells.  E** never goes to memory; f** = F**/E** is
// the reduced flux of the new state and goes straight to the output.
// The arithmetic is that of advect_block + freq_cell<float, float> step for
// step, so both paths give identical bits.
struct FusedSink {
  static constexpr bool kHeavy = true;      // elimination state of two cells across bins
  FreqCell<float, float> fc[2];
  float al[2], qp[2], Cp[2], ep[2];
  double acF[2];
  double f4[2][4];
  FreqRow row[2];

  __device__ __forceinline__ void init(const GridArgs<float>& a, const bool* own,
                                       const unsigned* cidx, const int* ccls) {
    const size_t nc = (size_t)a.nx * a.ny;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const size_t c = cidx[m];
      const int cl = ccls[m];
      al[m] = own[m] ? a.alpha[c] : 0.0f;
      acF[m] = own[m] ? (double)a.acF[c] : 0.0;
      FreqCell<float, float>& f = fc[m];
      f.gxx = own[m] ? a.grad[c] : 0.0f;
      f.gyy = own[m] ? a.grad[nc + c] : 0.0f;
      f.gxy = own[m] ? a.grad[2 * nc + c] : 0.0f;
      f.gpp = own[m] ? a.grad[3 * nc + c] : 0.0f;
      f.dd = (float)a.dD2h[cl] * al[m];
      f.hkT = (float)a.hkT[cl];
      f.recoil = a.recoil != 0;
      f.doppler = a.doppler != 0 &&
          ((f.gxx != 0.0f) || (f.gyy != 0.0f) || (f.gxy != 0.0f) || (f.gpp != 0.0f));
      qp[m] = Cp[m] = ep[m] = 0.0f;
      f4[m][0] = f4[m][1] = f4[m][2] = f4[m][3] = 0.0;
      row[m] = FreqRow();
    }
  }

  __device__ __forceinline__ void put(const GridArgs<float>& a, int m, int k, size_t koff,
                                      unsigned c, float h, float E, float X, float Y) {
    const size_t q = koff + c;
    float fxo, fyo;
    reduced_flux<float>(E, X, Y, fxo, fyo);
    __builtin_nontemporal_store(fxo, &a.fxo[q]);
    __builtin_nontemporal_store(fyo, &a.fyo[q]);
    float qk, Ck;
    fc[m].coeffs(a, k, h, fxo, fyo, qk, Ck);
    const double dn = a.dnu[k];
    const double aH = (double)al[m] * (double)h;
    const double aF = aH + acF[m];
    const double Xd = (double)fxo * (double)E, Yd = (double)fyo * (double)E;
    f4[m][0] += dn * aF * Xd;
    f4[m][1] += dn * aF * Yd;
    f4[m][2] += dn * aH * Xd;
    f4[m][3] += dn * aH * Yd;
    if (k > 0) {
      float gl, gr;
      if (qp[m] > 0.0f && qk > 0.0f) {
        interface_rates<float>(qp[m], Cp[m], qk, Ck, gl, gr);
      } else {
        gl = Cp[m] < 0.0f ? -Cp[m] : 0.0f;      // K -> 0: first-order upwind
        gr = Ck > 0.0f ? Ck : 0.0f;
      }
      const double ctdt = (double)a.ctdt;
      const double a_k = ctdt * (double)gl * a.inv_dnu[k - 1];
      const double b_next = ctdt * (double)gr * a.inv_dnu[k];
      const size_t nc = (size_t)a.nx * a.ny;
      row[m].eliminate<float>(k - 1, a.dnu[k - 1] * (double)ep[m], a_k, b_next, &a.zw[q - nc]);
    }
    qp[m] = qk;
    Cp[m] = Ck;
    ep[m] = E;
  }

  __device__ __forceinline__ void finish(const GridArgs<float>& a, const bool* own,
                                         const unsigned* cidx) {
    const size_t nc = (size_t)a.nx * a.ny;
    const int nb = a.nb;
#pragma unroll
    for (int m = 0; m < 2; ++m)
      if (own[m])
        row[m].eliminate<float>(nb - 1, a.dnu[nb - 1] * (double)ep[m], 0.0, 0.0,
                                &a.zw[(size_t)(nb - 1) * nc + cidx[m]]);
#pragma unroll
    for (int m = 0; m < 2; ++m)
      if (own[m]) freq_backward<float>(a, cidx[m], nc, a.Eo, a.zw);
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      if (!own[m]) continue;
      const size_t c = cidx[m];
      a.force[c] = f4[m][0];
      a.force[nc + c] = f4[m][1];
      a.force[2 * nc + c] = f4[m][2];
      a.force[3 * nc + c] = f4[m][3];
    }
  }
};

// Batched fused step: work item = one tile (all bins) of a grid.
// Four waves per SIMD (128 registers).
template <bool AB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
void k_step_fused_batched(const GridArgs<float>* __restrict__ args,
                                                            const int* __restrict__ par, int n,
                                                            int sp, const int* __restrict__ off) {
  __shared__ AdvShared<float> S;
  const int total = off[n];
  for (int w = (int)xcd_logical_block(); w < total; w += gridDim.x) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (off[mid] <= w) lo = mid; else hi = mid;
    }
    const GridArgs<float> a = global_args(args[((par[lo] ^ sp) & 1) * n + lo]);
    FusedSink sink;
    advect_block<float, 0, AB, false>(a, (unsigned)(w - off[lo]), S, sink);
  }
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
// Physical state out of the internal one: E_phys = 2^e2 E, F_phys = 2^e2 f E
// (product in double), for the w x h window (i0, j0) of every bin; the whole
// grid is the window (0, 0, nx, ny).  Null outputs are skipped.
template <typename S>
__global__ void k_state_out(const S* __restrict__ E, const S* __restrict__ fx,
                            const S* __restrict__ fy, int nx, int ny, int nb, int i0, int j0,
                            int w, int h, int e2, double* __restrict__ dE,
                            double* __restrict__ dFx, double* __restrict__ dFy) {
  const size_t per = (size_t)w * h, n = per * nb;
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (size_t)gridDim.x * blockDim.x) {
    const size_t k = q / per, r = q % per;
    const int jj = (int)(r / w), ii = (int)(r % w);
    const size_t src = (k * ny + j0 + jj) * nx + i0 + ii;
    const double e = (double)E[src];
    if (dE) dE[q] = ldexp(e, e2);
    if (dFx) dFx[q] = ldexp((double)fx[src] * e, e2);
    if (dFy) dFy[q] = ldexp((double)fy[src] * e, e2);
  }
}

// Internal state from the physical one: E = 2^e2 E_phys, f = F/E (0 where E <= 0).
template <typename D>
__global__ void k_state_in(const double* __restrict__ sE, const double* __restrict__ sFx,
                           const double* __restrict__ sFy, size_t n, int e2, D* __restrict__ E,
                           D* __restrict__ fx, D* __restrict__ fy) {
  for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (size_t)gridDim.x * blockDim.x) {
    const double e = sE[q];
    const bool pos = e > 0.0;
    E[q] = (D)ldexp(e, e2);
    fx[q] = pos ? (D)(sFx[q] / e) : D(0);
    fy[q] = pos ? (D)(sFy[q] / e) : D(0);
  }
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
constexpr int kBK = 28;   // bins per advection block (7 runs for 194 bins)

// Bin runs of the plain advection of one grid: 28 bins per block, or, on
// grids whose 28-bin launch is under two rounds of blocks (1024 slots at
// four waves per SIMD), 14 bins if that gives four rounds, else 7: at 64^2
// the kernel takes 30 instead of 92 us.  The bits do not depend on the run
// length.
constexpr unsigned kRoundsBlocks = 4096;
constexpr unsigned kFewBlocks = 2048;

template <typename R>
hipError_t launch_advect(const GridArgs<R>& a, hipStream_t s) {
  const unsigned nbx = (a.nx + kTX - 1) / kTX, nby = (a.ny + kTY - 1) / kTY;
  const unsigned nbz = (a.nb + kBK - 1) / kBK;
  const dim3 g(nbx * nby * nbz), b(256);
  if (a.flux) {                      // the eigenvalue HLL flux (no runtime controls)
    hipLaunchKernelGGL((k_advect_source<R, kBK, false, false, true>), g, b, 0, s, a);
    return hipGetLastError();
  }
  if (!a.substeps && !a.active && g.x < kFewBlocks) {
    const unsigned n14 = nbx * nby * ((a.nb + 13) / 14), n7 = nbx * nby * ((a.nb + 6) / 7);
    if (n14 >= kRoundsBlocks)
      hipLaunchKernelGGL((k_advect_source<R, 14, false, false>), dim3(n14), b, 0, s, a);
    else
      hipLaunchKernelGGL((k_advect_source<R, 7, false, false>), dim3(n7), b, 0, s, a);
    return hipGetLastError();
  }
  if (a.substeps) {
    if (a.active) hipLaunchKernelGGL((k_advect_source<R, kBK, true, true>), g, b, 0, s, a);
    else          hipLaunchKernelGGL((k_advect_source<R, kBK, false, true>), g, b, 0, s, a);
  } else {
    if (a.active) hipLaunchKernelGGL((k_advect_source<R, kBK, true, false>), g, b, 0, s, a);
    else          hipLaunchKernelGGL((k_advect_source<R, kBK, false, false>), g, b, 0, s, a);
  }
  return hipGetLastError();
}

template <typename R>
hipError_t launch_band_step(const GridArgs<R>& a, hipStream_t s) {
  const unsigned nbx = (a.nx + kTX - 1) / kTX, nby = (a.ny + kTY - 1) / kTY;
  hipLaunchKernelGGL((k_band_step<R>), dim3(nbx * nby), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_freq(const GridArgs<R>& a, hipStream_t s) {
  size_t nc = (size_t)a.nx * a.ny;
  const dim3 g((unsigned)((nc + 255) / 256));
  if (a.substeps) {
    hipLaunchKernelGGL((k_freq_sub<R, 0>), g, dim3(256), 0, s, a);
    if (sizeof(R) == 4 && a.islands) hipLaunchKernelGGL((k_freq_sub<R, 1>), g, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (nc < kTwoPhaseCells<R> && a.nb > 1) {
    const size_t nt = (size_t)(a.nb - 1) * nc;
    hipLaunchKernelGGL((k_freq_rates<R>), dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, a);
    hipLaunchKernelGGL((k_freq_solve<R>), g, dim3(256), 0, s, a);
  } else {
    hipLaunchKernelGGL((k_freq<R, 0>), g, dim3(256), 0, s, a);
  }
  if (sizeof(R) == 4 && a.islands) hipLaunchKernelGGL((k_freq<R, 1>), g, dim3(256), 0, s, a);
  return hipGetLastError();
}

// ------------------------------------------------------------ active bins
// Section 2.2 (active bins): bin k is advected when its energy in the
// volume, W_k = dnu_k sum_c dV_c E_k,c, exceeds active_frac sum_k W_k.  The
// sums are double and deterministic: fixed partial sums of kEnergyCells
// cells per block (k_bin_energy), then one block adds them in order and sets
// the flags (k_bin_select).  The FP32 state carries the scale 2^e2, which
// cancels in the ratio.
constexpr int kEnergyCells = 8192;

template <typename R>
__global__ __launch_bounds__(256) void k_bin_energy(const R* __restrict__ E, int nx, size_t nc,
                                                    const double* __restrict__ wx,
                                                    const double* __restrict__ wy,
                                                    double* __restrict__ part, int nchunk) {
  __shared__ double red[4];
  const int k = blockIdx.y, q = blockIdx.x;
  const size_t c0 = (size_t)q * kEnergyCells;
  const size_t c1 = c0 + kEnergyCells < nc ? c0 + kEnergyCells : nc;
  const R* Ek = E + (size_t)k * nc;
  size_t c = c0 + threadIdx.x;
  int j = (int)(c / (size_t)nx), i = (int)(c - (size_t)j * nx);
  auto next = [&](int& ii, int& jj) {     // the cell 256 further on
    ii += 256;
    while (ii >= nx) { ii -= nx; ++jj; }
  };
  // four cells 256 apart per iteration: four loads in flight, four sums
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (; c + 768 < c1; c += 1024) {
    int i1 = i, j1 = j;
    next(i1, j1);
    int i2 = i1, j2 = j1;
    next(i2, j2);
    int i3 = i2, j3 = j2;
    next(i3, j3);
    const double e0 = (double)Ek[c], e1 = (double)Ek[c + 256], e2 = (double)Ek[c + 512],
                 e3 = (double)Ek[c + 768];
    s0 += wx[i] * wy[j] * e0;
    s1 += wx[i1] * wy[j1] * e1;
    s2 += wx[i2] * wy[j2] * e2;
    s3 += wx[i3] * wy[j3] * e3;
    i = i3; j = j3;
    next(i, j);
  }
  for (; c < c1; c += 256) {
    s0 += wx[i] * wy[j] * (double)Ek[c];
    next(i, j);
  }
  double s = (s0 + s1) + (s2 + s3);
  // fixed-order reduction: within the wave, then the four waves in order
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[(size_t)k * nchunk + q] = ((red[0] + red[1]) + red[2]) + red[3];
}

// One block; dynamic LDS of nb doubles.
__global__ __launch_bounds__(256) void k_bin_select(const double* __restrict__ part, int nchunk,
                                                    int nb, const double* __restrict__ dnu,
                                                    double frac, int32_t* __restrict__ active) {
  extern __shared__ double W[];
  for (int k = threadIdx.x; k < nb; k += 256) {
    double s = 0.0;
    for (int q = 0; q < nchunk; ++q) s += part[(size_t)k * nchunk + q];
    W[k] = dnu[k] * s;
  }
  __syncthreads();
  double tot = 0.0;
  for (int k = 0; k < nb; ++k) tot += W[k];
  for (int k = threadIdx.x; k < nb; k += 256) active[k] = W[k] > frac * tot ? 1 : 0;
}

int energy_chunks(size_t nc) { return (int)((nc + kEnergyCells - 1) / kEnergyCells); }

template <typename R>
hipError_t launch_active_bins(const R* E, int nx, int ny, int nb, const double* wx,
                              const double* wy, const double* dnu, double frac, double* part,
                              int32_t* active, hipStream_t s) {
  const size_t nc = (size_t)nx * ny;
  const int nchunk = energy_chunks(nc);
  hipLaunchKernelGGL((k_bin_energy<R>), dim3(nchunk, nb), dim3(256), 0, s, E, nx, nc, wx, wy,
                     part, nchunk);
  hipLaunchKernelGGL(k_bin_select, dim3(1), dim3(256), nb * sizeof(double), s, part, nchunk, nb,
                     dnu, frac, active);
  return hipGetLastError();
}

int tile_count(int nx, int ny) { return ((nx + kTX - 1) / kTX) * ((ny + kTY - 1) / kTY); }
int advect_blocks(int nx, int ny, int nb, int bk) {
  return tile_count(nx, ny) * (bk > 0 ? (nb + bk - 1) / bk : 1);
}

int freq_blocks(int nx, int ny) { return (int)(((size_t)nx * ny + 255) / 256); }

const int kBatchBK[kNumBatchVariants] = {7, 14, 28, 49, -1};

template <typename R, bool AB>
hipError_t launch_advect_batched_ab(int variant, const GridArgs<R>* args, const int* par, int n,
                                    int sp, const int* off, int nblocks, hipStream_t s) {
  dim3 g(nblocks), b(256);
  switch (variant) {
    case 0: hipLaunchKernelGGL((k_advect_batched<R, 7, AB>), g, b, 0, s, args, par, n, sp, off); break;
    case 1: hipLaunchKernelGGL((k_advect_batched<R, 14, AB>), g, b, 0, s, args, par, n, sp, off); break;
    case 2: hipLaunchKernelGGL((k_advect_batched<R, 28, AB>), g, b, 0, s, args, par, n, sp, off); break;
    case 3: hipLaunchKernelGGL((k_advect_batched<R, 49, AB>), g, b, 0, s, args, par, n, sp, off); break;
    default:
      if constexpr (sizeof(R) == 4)
        hipLaunchKernelGGL(k_step_fused_batched<AB>, g, b, 0, s, (const GridArgs<float>*)args, par,
                           n, sp, off);
      else
        return hipErrorInvalidValue;              // fused: float storage only
      break;
  }
  return hipGetLastError();
}

template <typename R>
hipError_t launch_advect_batched(int variant, const GridArgs<R>* args, const int* par, int n,
                                 int sp, const int* off, int nblocks, int active, hipStream_t s) {
  return active ? launch_advect_batched_ab<R, true>(variant, args, par, n, sp, off, nblocks, s)
                : launch_advect_batched_ab<R, false>(variant, args, par, n, sp, off, nblocks, s);
}

template <typename R>
hipError_t launch_freq_batched(const GridArgs<R>* args, const int* par, int n, int sp,
                               const int* off, int nblocks, int islands, const int* offr,
                               int nrates, hipStream_t s) {
  if ((size_t)nblocks * 256 < kTwoPhaseCells<R>) {     // a batch of few cells
    if (nrates > 0)
      hipLaunchKernelGGL((k_freq_rates_batched<R>), dim3(nrates), dim3(256), 0, s, args, par, n,
                         sp, offr);
    hipLaunchKernelGGL((k_freq_solve_batched<R>), dim3(nblocks), dim3(256), 0, s, args, par, n,
                       sp, off);
    if (sizeof(R) == 4 && islands)
      hipLaunchKernelGGL((k_freq_batched<R, 1>), dim3(nblocks), dim3(256), 0, s, args, par, n, sp,
                         off);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((k_freq_batched<R, 0>), dim3(nblocks), dim3(256), 0, s, args, par, n, sp, off);
  if (sizeof(R) == 4 && islands)
    hipLaunchKernelGGL((k_freq_batched<R, 1>), dim3(nblocks), dim3(256), 0, s, args, par, n, sp, off);
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

template <typename S>
hipError_t launch_state_out(const S* E, const S* fx, const S* fy, int nx, int ny, int nb, int i0,
                            int j0, int w, int h, int e2, double* dE, double* dFx, double* dFy,
                            hipStream_t s) {
  const size_t n = (size_t)w * h * nb;
  unsigned g = (unsigned)std::min<size_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL((k_state_out<S>), dim3(g ? g : 1), dim3(256), 0, s, E, fx, fy, nx, ny, nb,
                     i0, j0, w, h, e2, dE, dFx, dFy);
  return hipGetLastError();
}
template <typename D>
hipError_t launch_state_in(const double* sE, const double* sFx, const double* sFy, size_t n,
                           int e2, D* E, D* fx, D* fy, hipStream_t s) {
  unsigned g = (unsigned)std::min<size_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL((k_state_in<D>), dim3(g ? g : 1), dim3(256), 0, s, sE, sFx, sFy, n, e2, E, fx,
                     fy);
  return hipGetLastError();
}
template hipError_t launch_state_out<float>(const float*, const float*, const float*, int, int, int,
                                            int, int, int, int, int, double*, double*, double*,
                                            hipStream_t);
template hipError_t launch_state_out<double>(const double*, const double*, const double*, int, int,
                                             int, int, int, int, int, int, double*, double*,
                                             double*, hipStream_t);
template hipError_t launch_state_in<float>(const double*, const double*, const double*, size_t, int,
                                           float*, float*, float*, hipStream_t);
template hipError_t launch_state_in<double>(const double*, const double*, const double*, size_t,
                                            int, double*, double*, double*, hipStream_t);

hipError_t launch_force_out(const double* force, size_t nc, int e2, double* fx, double* fy,
                            double* gx, double* gy, hipStream_t s) {
  unsigned g = (unsigned)std::min<size_t>((nc + 255) / 256, 65536);
  hipLaunchKernelGGL(k_force_out, dim3(g ? g : 1), dim3(256), 0, s, force, nc, e2, fx, fy, gx, gy);
  return hipGetLastError();
}

template hipError_t launch_step<float>(const GridArgs<float>&, hipStream_t);
template hipError_t launch_step<double>(const GridArgs<double>&, hipStream_t);
template hipError_t launch_advect_batched<float>(int, const GridArgs<float>*, const int*, int, int, const int*, int, int, hipStream_t);
template hipError_t launch_advect_batched<double>(int, const GridArgs<double>*, const int*, int, int, const int*, int, int, hipStream_t);
template hipError_t launch_freq_batched<float>(const GridArgs<float>*, const int*, int, int, const int*, int, int, const int*, int, hipStream_t);
template hipError_t launch_freq_batched<double>(const GridArgs<double>*, const int*, int, int, const int*, int, int, const int*, int, hipStream_t);
template hipError_t launch_band_step<float>(const GridArgs<float>&, hipStream_t);
template hipError_t launch_band_step<double>(const GridArgs<double>&, hipStream_t);
template hipError_t launch_advect<float>(const GridArgs<float>&, hipStream_t);
template hipError_t launch_advect<double>(const GridArgs<double>&, hipStream_t);
template hipError_t launch_freq<float>(const GridArgs<float>&, hipStream_t);
template hipError_t launch_active_bins<float>(const float*, int, int, int, const double*,
                                              const double*, const double*, double, double*,
                                              int32_t*, hipStream_t);
template hipError_t launch_active_bins<double>(const double*, int, int, int, const double*,
                                               const double*, const double*, double, double*,
                                               int32_t*, hipStream_t);
template hipError_t launch_freq<double>(const GridArgs<double>&, hipStream_t);
template hipError_t launch_residual<float>(const float*, const float*, size_t, double*, int, double*, hipStream_t);
template hipError_t launch_residual<double>(const double*, const double*, size_t, double*, int, double*, hipStream_t);

}  // namespace m1
