// Set-up kernels (run once per m1_init): bin-averaged Voigt profiles per
// temperature class, per-cell opacities, velocity gradients, and the
// reductions behind the CFL time step.
#include "m1_kernels.h"
#include "m1_dawson.h"

namespace m1 {

// I(x_hi, a) - I(x_lo, a) for the second-order Voigt expansion
// I(x, a) = sqrt(pi)/2 erf(x) - (2a/sqrt(pi)) Dawson(x) + a^2 x exp(-x^2)
// (Appendix A).  The erf difference goes through erfc on either side of the
// line centre so that far-wing bins keep their digits.
__device__ double voigt_I_diff(double lo, double hi, double a, const double* nodes) {
  const double sqpi = 1.77245385090551602729816748334;
  double ep;
  if (lo >= 0.0) ep = erfc(lo) - erfc(hi);
  else if (hi <= 0.0) ep = erfc(-hi) - erfc(-lo);
  else ep = erf(hi) - erf(lo);
  double dw = dawson(hi, nodes) - dawson(lo, nodes);
  return 0.5 * sqpi * ep - (2.0 * a / sqpi) * dw +
         a * a * (hi * exp(-hi * hi) - lo * exp(-lo * lo));
}

__global__ void k_class_voigt(const double* __restrict__ dnuD, const double* __restrict__ av,
                              int64_t ncls, const double* __restrict__ edges,
                              const double* __restrict__ dnu, int nb,
                              const double* __restrict__ nodes, double* __restrict__ out) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ncls * nb) return;
  int64_t cl = t / nb;
  int k = (int)(t - cl * nb);
  double dD = dnuD[cl];
  double lo = edges[k] / dD, hi = edges[k + 1] / dD;
  out[t] = voigt_I_diff(lo, hi, av[cl], nodes) / (dnu[k] / dD);
}

template <typename R>
__global__ void k_class_norm(const double* __restrict__ hb, int64_t ncls,
                             const double* __restrict__ dnu, int nb, R* __restrict__ hbar,
                             R* __restrict__ phi) {
  int64_t cl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cl >= ncls) return;
  const double* h = hb + cl * nb;
  double s = 0.0;
  for (int k = 0; k < nb; ++k) s += dnu[k] * h[k];
  for (int k = 0; k < nb; ++k) {
    hbar[cl * nb + k] = (R)h[k];
    phi[cl * nb + k] = (R)(h[k] / s);
  }
}

template <typename R>
hipError_t launch_class_profiles(const double* dnuD, const double* av, int64_t ncls,
                                 const double* dnu_edges, const double* dnu, int nb,
                                 const double* nodes, double* tmp, R* hbar, R* phi,
                                 hipStream_t s) {
  int64_t n = ncls * nb;
  hipLaunchKernelGGL(k_class_voigt, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dnuD,
                     av, ncls, dnu_edges, dnu, nb, nodes, tmp);
  hipLaunchKernelGGL((k_class_norm<R>), dim3((unsigned)((ncls + 255) / 256)), dim3(256), 0, s,
                     tmp, ncls, dnu, nb, hbar, phi);
  return hipGetLastError();
}

// Line-centre cross-section 5.9e-14 (T/1e4 K)^-1/2 cm^2 (Section 2.1).
template <typename R>
__global__ void k_cell_setup(CellInputs in, size_t nc, double dmin, double fp64_tau, int e2,
                             R* alpha, R* acF, R* acabs, R* pda, R* em, uint8_t* island) {
  size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  double a = in.n_HI[c] * (5.9e-14 / sqrt(in.T[c] / 1.0e4));
  alpha[c] = (R)a;
  acF[c] = (R)in.acF[c];
  acabs[c] = (R)in.acabs[c];
  pda[c] = (R)(in.pd[c] * a);
  em[c] = (R)(ldexp(in.emis[c], e2) / kC);
  island[c] = (a * dmin >= fp64_tau) ? 1 : 0;
}

template <typename R>
hipError_t launch_cell_setup(const CellInputs& in, size_t nc, double dmin, double fp64_tau,
                             int e2, R* alpha, R* acF, R* acabs, R* pda, R* em,
                             uint8_t* island, hipStream_t s) {
  hipLaunchKernelGGL((k_cell_setup<R>), dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s, in,
                     nc, dmin, fp64_tau, e2, alpha, acF, acabs, pda, em, island);
  return hipGetLastError();
}

// Face mean velocities.  Ghost velocity: copy at vacuum boundaries, mirror
// (normal component negated) at reflecting ones.  x-faces: f in [0, nx],
// tmp layout [unx | utx | uny | uty].
__global__ void k_face_velocity(CellInputs in, int nx, int ny, int bc0, int bc1, int bc2,
                                int bc3, double* __restrict__ tmp) {
  size_t nfx = (size_t)(nx + 1) * ny, nfy = (size_t)nx * (ny + 1);
  size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double* unx = tmp;
  double* utx = tmp + nfx;
  double* uny = tmp + 2 * nfx;
  double* uty = tmp + 2 * nfx + nfy;
  if (t < nfx) {
    int j = (int)(t / (nx + 1)), f = (int)(t % (nx + 1));
    int il = f - 1, ir = f;
    double uxl, uyl, uxr, uyr;
    if (il < 0) {
      size_t c = (size_t)j * nx;
      uxl = (bc0 == kReflect) ? -in.ux[c] : in.ux[c];
      uyl = in.uy[c];
    } else { size_t c = (size_t)j * nx + il; uxl = in.ux[c]; uyl = in.uy[c]; }
    if (ir >= nx) {
      size_t c = (size_t)j * nx + nx - 1;
      uxr = (bc1 == kReflect) ? -in.ux[c] : in.ux[c];
      uyr = in.uy[c];
    } else { size_t c = (size_t)j * nx + ir; uxr = in.ux[c]; uyr = in.uy[c]; }
    unx[t] = 0.5 * (uxl + uxr);
    utx[t] = 0.5 * (uyl + uyr);
  } else if (t < nfx + nfy) {
    size_t u = t - nfx;
    int f = (int)(u / nx), i = (int)(u % nx);
    int jl = f - 1, jr = f;
    double uxl, uyl, uxr, uyr;
    if (jl < 0) {
      size_t c = (size_t)i;
      uyl = (bc2 == kReflect) ? -in.uy[c] : in.uy[c];
      uxl = in.ux[c];
    } else { size_t c = (size_t)jl * nx + i; uxl = in.ux[c]; uyl = in.uy[c]; }
    if (jr >= ny) {
      size_t c = (size_t)(ny - 1) * nx + i;
      uyr = (bc3 == kReflect) ? -in.uy[c] : in.uy[c];
      uxr = in.ux[c];
    } else { size_t c = (size_t)jr * nx + i; uxr = in.ux[c]; uyr = in.uy[c]; }
    uny[u] = 0.5 * (uyl + uyr);
    uty[u] = 0.5 * (uxl + uxr);
  }
}

// Cell velocity gradients from face means (Appendix A):
// d u/dx = (u_{i+1/2} - u_{i-1/2})/(x_{i+1/2} - x_{i-1/2}),
// <u_R/R> = (u_{R,i+1/2} + u_{R,i-1/2})/(R_{i+1/2} + R_{i-1/2}).
template <typename R>
__global__ void k_gradients(int nx, int ny, int geom, const double* __restrict__ xe,
                            const double* __restrict__ ye, const double* __restrict__ tmp,
                            R* __restrict__ ufx, R* __restrict__ ufy, R* __restrict__ grad) {
  size_t nfx = (size_t)(nx + 1) * ny, nfy = (size_t)nx * (ny + 1), nc = (size_t)nx * ny;
  const double* unx = tmp;
  const double* utx = tmp + nfx;
  const double* uny = tmp + 2 * nfx;
  const double* uty = tmp + 2 * nfx + nfy;
  size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nfx) ufx[t] = (R)unx[t];
  if (t < nfy) ufy[t] = (R)uny[t];
  if (t >= nc) return;
  int j = (int)(t / nx), i = (int)(t % nx);
  size_t fm = (size_t)j * (nx + 1) + i, fp = fm + 1;
  double hx = xe[i + 1] - xe[i];
  double dxux = (unx[fp] - unx[fm]) / hx;
  double dxuy = (utx[fp] - utx[fm]) / hx;
  double uRR = (geom == 1) ? (unx[fp] + unx[fm]) / (xe[i + 1] + xe[i]) : 0.0;
  size_t gm = (size_t)j * nx + i, gp = gm + nx;
  double hy = ye[j + 1] - ye[j];
  double dyuy = (uny[gp] - uny[gm]) / hy;
  double dyux = (uty[gp] - uty[gm]) / hy;
  grad[t] = (R)dxux;
  grad[nc + t] = (R)dyuy;
  grad[2 * nc + t] = (R)(dyux + dxuy);
  grad[3 * nc + t] = (R)uRR;
}

template <typename R>
hipError_t launch_velocity(const CellInputs& in, int nx, int ny, int geom, const int* bc,
                           const double* xe, const double* ye, double* tmp, R* ufx, R* ufy,
                           R* grad, hipStream_t s) {
  size_t nfx = (size_t)(nx + 1) * ny, nfy = (size_t)nx * (ny + 1);
  size_t n1 = nfx + nfy;
  hipLaunchKernelGGL(k_face_velocity, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, s, in,
                     nx, ny, bc[0], bc[1], bc[2], bc[3], tmp);
  size_t n2 = std::max(std::max(nfx, nfy), (size_t)nx * ny);
  hipLaunchKernelGGL((k_gradients<R>), dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, nx,
                     ny, geom, xe, ye, (const double*)tmp, ufx, ufy, grad);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_init_reduce(CellInputs in, size_t nc,
                                                     double* __restrict__ partial) {
  __shared__ double su[256], se[256], st[256];
  double umax = 0.0, emax = 0.0, tmin = 1.0e300;
  for (size_t c = (size_t)blockIdx.x * 256 + threadIdx.x; c < nc; c += (size_t)gridDim.x * 256) {
    double u = sqrt(in.ux[c] * in.ux[c] + in.uy[c] * in.uy[c]);
    umax = u > umax ? u : umax;
    emax = in.emis[c] > emax ? in.emis[c] : emax;
    tmin = in.T[c] < tmin ? in.T[c] : tmin;
  }
  su[threadIdx.x] = umax; se[threadIdx.x] = emax; st[threadIdx.x] = tmin;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      su[threadIdx.x] = fmax(su[threadIdx.x], su[threadIdx.x + w]);
      se[threadIdx.x] = fmax(se[threadIdx.x], se[threadIdx.x + w]);
      st[threadIdx.x] = fmin(st[threadIdx.x], st[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[3 * blockIdx.x] = su[0];
    partial[3 * blockIdx.x + 1] = se[0];
    partial[3 * blockIdx.x + 2] = st[0];
  }
}

hipError_t launch_init_reduce(const CellInputs& in, size_t nc, double* partial, int nblk,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_init_reduce, dim3(nblk), dim3(256), 0, s, in, nc, partial);
  return hipGetLastError();
}

// Dynamic reduced speed of light (Section 2.1): block maxima over the cells
// of max[1, (a_v tau_0)^(1/3) f_abs] max(|u|, c_s), with tau_0 and tau_c the
// line-centre and continuum-absorption depths over the larger cell side dmax
// and f_abs = 1 / (1 + (a_v tau_0)^(1/3) tau_c + 0.6 p_d tau_0).  A maximum
// does not depend on the order of the reduction.  A cell whose term is not a
// number (T <= 0, a negative depth) makes the block's result NaN, which the
// host reports.
__device__ __forceinline__ double nan_max(double a, double b) {
  return (a != a || b != b) ? __builtin_nan("") : fmax(a, b);
}

__global__ __launch_bounds__(256) void k_dyn_rsl(CellInputs in, const double* __restrict__ cs,
                                                 size_t nc, double dmax,
                                                 double* __restrict__ partial) {
  __shared__ double sm[256];
  double best = 0.0;
  for (size_t c = (size_t)blockIdx.x * 256 + threadIdx.x; c < nc; c += (size_t)gridDim.x * 256) {
    const double t4 = sqrt(in.T[c] / 1.0e4);
    const double tau0 = in.n_HI[c] * (5.9e-14 / t4) * dmax;
    const double tauc = in.acabs[c] * dmax;
    const double at = cbrt((4.7e-4 / t4) * tau0);
    const double fabs_ = 1.0 / (1.0 + at * tauc + 0.6 * in.pd[c] * tau0);
    const double u = sqrt(in.ux[c] * in.ux[c] + in.uy[c] * in.uy[c]);
    const double term = nan_max(1.0, at * fabs_) * nan_max(u, cs[c]);
    best = nan_max(best, term);
  }
  sm[threadIdx.x] = best;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sm[threadIdx.x] = nan_max(sm[threadIdx.x], sm[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sm[0];
}

hipError_t launch_dyn_rsl(const CellInputs& in, const double* cs, size_t nc, double dmax,
                          double* partial, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(k_dyn_rsl, dim3(nblk), dim3(256), 0, s, in, cs, nc, dmax, partial);
  return hipGetLastError();
}

// The maximum of n block maxima (NaN if any is NaN) into *out, one block.
__global__ __launch_bounds__(256) void k_max_of(const double* __restrict__ partial, int n,
                                                double* __restrict__ out) {
  __shared__ double sm[256];
  double best = 0.0;
  for (int b = threadIdx.x; b < n; b += 256) best = nan_max(best, partial[b]);
  sm[threadIdx.x] = best;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sm[threadIdx.x] = nan_max(sm[threadIdx.x], sm[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sm[0];
}

hipError_t launch_max_of(const double* partial, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_max_of, dim3(1), dim3(256), 0, s, partial, n, out);
  return hipGetLastError();
}

template hipError_t launch_class_profiles<float>(const double*, const double*, int64_t,
                                                 const double*, const double*, int,
                                                 const double*, double*, float*, float*,
                                                 hipStream_t);
template hipError_t launch_class_profiles<double>(const double*, const double*, int64_t,
                                                  const double*, const double*, int,
                                                  const double*, double*, double*, double*,
                                                  hipStream_t);
template hipError_t launch_cell_setup<float>(const CellInputs&, size_t, double, double, int,
                                             float*, float*, float*, float*, float*, uint8_t*,
                                             hipStream_t);
template hipError_t launch_cell_setup<double>(const CellInputs&, size_t, double, double, int,
                                              double*, double*, double*, double*, double*,
                                              uint8_t*, hipStream_t);
template hipError_t launch_velocity<float>(const CellInputs&, int, int, int, const int*,
                                           const double*, const double*, double*, float*,
                                           float*, float*, hipStream_t);
template hipError_t launch_velocity<double>(const CellInputs&, int, int, int, const int*,
                                            const double*, const double*, double*, double*,
                                            double*, double*, hipStream_t);

}  // namespace m1
