// Device-side building blocks of the M1 Lyman-alpha step (gfx950).
//
// Everything here is written for CDNA wave64 execution: one lane per cell
// (advection: one cell and a run of bins; frequency step: one cell, all
// bins), coalesced along x of the [bin][y][x] structure-of-arrays state.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace m1 {

constexpr double kC = 2.99792458e10;        // speed of light [cm/s]
constexpr int kVacuum = 0;
constexpr int kReflect = 1;

// Frequency-step scratch of one cell and bin: z_k = d_k/p_k, w_k = b_{k+1}/p_k
// (stored together so each is one 8- or 16-byte access).
template <typename R>
struct __attribute__((aligned(2 * sizeof(R)))) ZW {
  R z, w;
};

// Kernel arguments of one grid.  Pointers are into the handle's workspace.
template <typename R>
struct GridArgs {
  int nx, ny, nb, geom;
  int bc[4];
  int recoil, doppler;
  int islands;            // FP32 storage with a finite fp64_tau: island cells may exist
  R ctdt;                 // c_tilde * dt
  R ctdt_c;               // c_tilde * dt / c (work term)
  // ping-pong state: in -> out.  The state of a cell and bin is E and the
  // reduced flux f = F/E (0 where E = 0): the frequency step changes E only,
  // since its rescale F -> F E^{n+1}/E** leaves F/E as it is.
  const R *E, *fx, *fy;
  R *Eo, *fxo, *fyo;
  // per cell
  const int32_t *cls;
  const uint8_t *island;
  const R *alpha, *acF, *acabs, *pda, *em;
  const R *grad;          // [4][ncell]: dx ux, dy uy, dy ux + dx uy, <u_R/R>
  const R *ufx, *ufy;     // face-normal velocities [(nx+1) ny], [nx (ny+1)]
  // per class and bin
  const R *hbar, *phi;    // [ncls][nb]
  const double *dD2h;     // [ncls] 0.5 dnu_D^2
  const double *hkT;      // [ncls] h / (k_B T)
  const double *dnu;      // [nb] bin widths
  const double *inv_dnu;  // [nb] 1 / bin widths
  const double *two_nu;   // [nb] 2 / nu_k
  const double *nu_c;     // [nb] nu_k / c
  // geometry per column (index i + 2, i in [-2, nx+1]) and per row
  const R *xidl, *xhm, *xhp;   // 1/(xc_i - xc_{i-1}), x_{i-1/2} - xc_i, x_{i+1/2} - xc_i
  const R *cxm, *cxp, *chp;    // [nx] ctdt A_{i-1/2}/dV, ctdt A_{i+1/2}/dV, ctdt (A+ - A-)/dV
  const R *yidl, *yhm, *yhp;
  const R *cy;                 // [ny] ctdt / dz_j
  // frequency step
  ZW<R> *zw;              // scratch [nb][ncell]
  double *force;          // [4][ncell]
  // active bins: flags [nb] of the bins this step advects (nullptr: all)
  const int32_t *active;
  // emission/absorption in substeps under the 10 % energy rule (0/1), and the
  // energy-density floor of the rule in state units
  int substeps;
  double e_floor;
  // interface flux: 0 corrected GLF (signal speeds -+c_tilde), 1 HLL with the
  // M1 system's eigenvalue signal speeds
  int flux;
  // broad bands (a grid of bands instead of line bins): per band and cell
  // [nb][ncell], absorption and flux opacities and the emission term L/c
  // (state units); nullptr for line grids
  const R *kabs, *kflux, *jsrc;
};

// Address-space hints for pointers read from a descriptor table in memory
// (batches).  Such pointers are generic: the compiler emits flat loads and
// stores through them, and vector loads even where the index is uniform.
// An empty move in the target address space (which the optimiser cannot fold
// away) restores what a kernel argument would tell it.  The pointer must be
// uniform across the wave: it is held in scalar registers.
//
// global_ptr: global memory (state, scratch, force).
template <typename T>
__device__ __forceinline__ T* global_ptr(T* p) {
  typedef __attribute__((address_space(1))) T* gptr;
  gptr g = (gptr)p;
  asm("" : "+s"(g));
  return (T*)g;
}

// const_ptr: memory that no kernel of the step writes (cell data, profiles,
// bin and geometry tables), so loads at a uniform index become scalar loads.
template <typename T>
__device__ __forceinline__ const T* const_ptr(const T* p) {
  typedef __attribute__((address_space(4))) const T* cptr;
  cptr g = (cptr)p;
  asm("" : "+s"(g));
  return (const T*)g;
}

// A grid's arguments read from a descriptor table, with these hints.
template <typename R>
__device__ __forceinline__ GridArgs<R> global_args(const GridArgs<R>& s) {
  GridArgs<R> a = s;
  a.E = global_ptr(a.E); a.fx = global_ptr(a.fx); a.fy = global_ptr(a.fy);
  a.Eo = global_ptr(a.Eo); a.fxo = global_ptr(a.fxo); a.fyo = global_ptr(a.fyo);
  a.zw = global_ptr(a.zw); a.force = global_ptr(a.force);
  a.cls = const_ptr(a.cls); a.island = const_ptr(a.island);
  a.alpha = const_ptr(a.alpha); a.acF = const_ptr(a.acF); a.acabs = const_ptr(a.acabs);
  a.pda = const_ptr(a.pda); a.em = const_ptr(a.em); a.grad = const_ptr(a.grad);
  a.ufx = const_ptr(a.ufx); a.ufy = const_ptr(a.ufy);
  a.hbar = const_ptr(a.hbar); a.phi = const_ptr(a.phi);
  a.dD2h = const_ptr(a.dD2h); a.hkT = const_ptr(a.hkT); a.dnu = const_ptr(a.dnu);
  a.inv_dnu = const_ptr(a.inv_dnu); a.two_nu = const_ptr(a.two_nu); a.nu_c = const_ptr(a.nu_c);
  a.xidl = const_ptr(a.xidl); a.xhm = const_ptr(a.xhm); a.xhp = const_ptr(a.xhp);
  a.cxm = const_ptr(a.cxm); a.cxp = const_ptr(a.cxp); a.chp = const_ptr(a.chp);
  a.yidl = const_ptr(a.yidl); a.yhm = const_ptr(a.yhm); a.yhp = const_ptr(a.yhp);
  a.cy = const_ptr(a.cy);
  a.active = const_ptr(a.active);
  a.kabs = const_ptr(a.kabs); a.kflux = const_ptr(a.kflux); a.jsrc = const_ptr(a.jsrc);
  return a;
}

// ---------------------------------------------------------------------------
// Levermore closure in cancellation-free form.  With f = |F|/E and
// s = sqrt(4 - 3 f^2):  (1 - chi)/2 = (1 - f^2)/(1 + s) = (s - 1)/3 (since
// s^2 - 1 = 3 (1 - f^2)) and (3 chi - 1)/2 h_i h_j = 3 f_i f_j / (2 + s), so
//   D = (s - 1)/3 I + 3 f (x) f / (2 + s),
// which needs no division by |F|, stays exact at F = 0, and needs a single
// reciprocal.  s - 1 is formed exactly from the rounded s (s in [1, 2]), so
// the isotropic part carries an absolute error of the order of the rounding
// of s, negligible against the free-streaming part as f -> 1.
template <typename R>
struct Eddington {
  R xx, yy, xy, pp;
};

// Reciprocal, square root and reciprocal square root.  Float: the hardware's
// 1-ulp instructions, used only on arguments that are normal numbers by
// construction.  Double reciprocal and square root: the hardware's
// approximations refined by two Newton steps (quadratic convergence, so the
// result is within about an ulp, though not correctly rounded), half the
// instructions of the IEEE sequences, which also handle scaling and special
// values that cannot occur here: the reciprocals are taken of normal numbers
// (quantities >= 0.2, or energies above recip_floor) and the square root of
// 4 - 3 f^2 in [1, 4].  The double reciprocal square root (rare branches
// only) stays IEEE.
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double frcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
// sqrt(a) = a / sqrt(a): Newton steps on g ~ sqrt(a) and h ~ 1 / (2 sqrt(a))
// from the hardware's 1/sqrt(a), then a last correction of g by its residual.
__device__ __forceinline__ double fsqrt(double a) {
  const double y = __builtin_amdgcn_rsq(a);
  double g = a * y, h = 0.5 * y;
  double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  const double d = fma(-g, g, a);
  return fma(d, h, g);
}
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double frsq(double x) { return 1.0 / sqrt(x); }

// min(q, 1) for q >= 0: one v_med3_f32 in float (median of q, 1 and 0), where
// fmin would also canonicalise its argument.
__device__ __forceinline__ float clamp_unit(float q) {
  return __builtin_amdgcn_fmed3f(q, 1.0f, 0.0f);
}
__device__ __forceinline__ double clamp_unit(double q) { return fmin(q, 1.0); }

template <typename R>
__device__ __forceinline__ Eddington<R> closure_f(R fx, R fy) {
  const R xx2 = fx * fx, yy2 = fy * fy;
  const R f2 = clamp_unit(xx2 + yy2);
  const R s = fsqrt(R(4) - R(3) * f2);    // in [1, 2]
  const R g = R(3) * frcp(R(2) + s);
  const R iso = (s - R(1)) * R(1.0 / 3.0);
  Eddington<R> d;
  d.xx = iso + g * xx2;
  d.yy = iso + g * yy2;
  d.xy = g * fx * fy;
  d.pp = iso;
  return d;
}

// Smallest E whose reciprocal is finite with margin (2^-120 in float,
// 2^-1000 in double).  Below it (subnormal far-wing values) f = F/E is formed
// by true division, which stays bounded because |F| <= E.
template <typename R>
__device__ __forceinline__ R recip_floor() {
  return sizeof(R) == 4 ? R(7.52316384526264e-37) : R(9.332636185032189e-302);
}

// The parts of the closure a face and a cell update need, from the squares
// of the components of a reduced flux with |f| <= 1 (f2 = fx^2 + fy^2):
// s = sqrt(4 - 3 f2), g = 3/(2 + s) formed as 1/(s/3 + 2/3) (one fused
// multiply-add and a reciprocal), iso = (s - 1)/3.  Then
// D = iso I + g f (x) f, D_phiphi = iso.
template <typename R>
struct ClosureParts {
  R s, g, iso;
};
template <typename R>
__device__ __forceinline__ ClosureParts<R> closure_parts(R f2) {
  ClosureParts<R> c;
  c.s = fsqrt(R(4) - R(3) * clamp_unit(f2));
  c.g = frcp(c.s * R(1.0 / 3.0) + R(2.0 / 3.0));
  c.iso = (c.s - R(1)) * R(1.0 / 3.0);
  return c;
}

// Reduced flux f = F/E (0 where E <= 0).
template <typename R>
__device__ __forceinline__ void reduced_flux(R E, R Fx, R Fy, R& fx, R& fy) {
  const bool big = E >= recip_floor<R>();
  const R inv = frcp(big ? E : R(1));
  fx = big ? Fx * inv : R(0);
  fy = big ? Fy * inv : R(0);
  if (!big && E > R(0)) {            // subnormal far-wing values only
    fx = Fx / E;
    fy = Fy / E;
  }
}

// Closure of a reduced flux, |f| > 1 scaled back to 1 first.
template <typename R>
__device__ __forceinline__ Eddington<R> closure_reduced(R fx, R fy) {
  const R n2 = fx * fx + fy * fy;
  const R sc = n2 > R(1) ? frsq(n2) : R(1);
  return closure_f(fx * sc, fy * sc);
}

// Scale s in (0, 1] with |s F| <= E for E > 0 (the causality condition
// |H|/J <= 1).  The squares of tiny components underflow in float below
// ~1e-19 (and in double below ~1e-154), which would hide a violation, so
// small E is checked after an exact rescaling: in float by the power of two
// that brings the largest of E, |X|, |Y| into [1/2, 1) (the squares of the
// rescaled values cannot overflow, and one that underflows is negligible
// against the largest), in double by 2^400.
template <typename R>
__device__ __forceinline__ R causal_scale(R E, R X, R Y) {
  const R tiny = sizeof(R) == 4 ? R(1e-18) : R(1e-150);
  if (E >= tiny) {
    const R q2 = X * X + Y * Y;
    R sc = R(1);
    if (q2 > E * E) sc = E * frsq(q2);      // rare: branch, not select
    return sc;
  }
  if constexpr (sizeof(R) == 4) {
    const float m = fmaxf(E, fmaxf(fabsf(X), fabsf(Y)));
    const int ex = __builtin_amdgcn_frexp_expf(m);
    const float e = __builtin_ldexpf(E, -ex), x = __builtin_ldexpf(X, -ex),
                y = __builtin_ldexpf(Y, -ex);
    const float q2 = x * x + y * y;
    return q2 > e * e ? e * frsq(q2) : 1.0f;
  } else {
    const double e = E * 0x1p400, x = X * 0x1p400, y = Y * 0x1p400;
    const double q2 = x * x + y * y;
    return q2 > e * e ? e / sqrt(q2) : 1.0;
  }
}

// MinMod limiter: the argument of smaller magnitude when a and b share a
// sign, else 0 -- which is exactly the median of (a, b, 0).  Float: one
// v_med3_f32.  Double: max(min(a,b),0) + min(max(a,b),0), where one of the
// two terms is always zero, so the sum is exact.
__device__ __forceinline__ float minmod(float a, float b) {
  return __builtin_amdgcn_fmed3f(a, b, 0.0f);
}
__device__ __forceinline__ double minmod(double a, double b) {
  return fmax(fmin(a, b), 0.0) + fmin(fmax(a, b), 0.0);
}

}  // namespace m1
