// C ABI of the M1 Lyman-alpha step: validation, workspace layout, set-up and
// the stepping / steady-state / output entry points declared in m1lya.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "m1lya.h"
#include "m1_dawson.h"
#include "m1_kernels.h"

using namespace m1;

namespace {

// Physical constants (cgs)
constexpr double kKB = 1.380649e-16;
constexpr double kHP = 6.62607015e-27;
constexpr double kMH = 1.6735575e-24;
constexpr double kLyaLambda = 1215.67e-8;
constexpr double kEV = 1.602176634e-12;
constexpr double kLyCeV = 13.6057;
constexpr double kPi = 3.14159265358979323846;
constexpr double kSqrtPi = 1.77245385090551602729816748334;

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess)                                                         \
      return fail(M1_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));     \
  } while (0)

double nu_lya() { return kC / kLyaLambda; }
double doppler_width(double T) { return nu_lya() * sqrt(2.0 * kKB * T / (kMH * kC * kC)); }

// Frequency grid of Section 2.1: symmetric in dnu = nu - nu_Lya, two central
// bins of width dnu_D(T_min), widths growing by q outward, half-width
// min(half_width dnu_D(T_min), 0.99 nu_Lya, nu_LyC - nu_Lya), last bin clipped.
struct FreqGrid {
  std::vector<double> edges;   // relative to nu_Lya, nb+1
  std::vector<double> dnu, nuc;
  int nb = 0;
};

int build_grid(const m1_config& c, FreqGrid& g) {
  if (!(c.T_min > 0) || !(c.q > 1.0) || !(c.half_width > 0))
    return fail(M1_EINVAL, "frequency grid needs T_min > 0, q > 1, half_width > 0");
  double w0 = doppler_width(c.T_min);
  double nuL = nu_lya();
  double X = std::min(std::min(c.half_width * w0, 0.99 * nuL), kLyCeV * kEV / kHP - nuL);
  std::vector<double> pos(1, 0.0);
  double s = 0.0, w = w0;
  while (s < X) {
    s += w;
    pos.push_back(s);
    w *= c.q;
    if (pos.size() > 100000) return fail(M1_EINVAL, "frequency grid too large");
  }
  pos.back() = X;
  int m = (int)pos.size() - 1;
  g.nb = 2 * m;
  g.edges.resize(g.nb + 1);
  for (int i = 0; i <= m; ++i) {
    g.edges[m + i] = pos[i];
    g.edges[m - i] = -pos[i];
  }
  g.dnu.resize(g.nb);
  g.nuc.resize(g.nb);
  for (int k = 0; k < g.nb; ++k) {
    g.dnu[k] = g.edges[k + 1] - g.edges[k];
    g.nuc[k] = nuL + 0.5 * (g.edges[k] + g.edges[k + 1]);
  }
  return M1_OK;
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  size_t state[2][3];
  size_t zw, force;
  size_t cls, island, alpha, acF, acabs, pda, em, grad, ufx, ufy;
  size_t hbar, phi, dD2h, hkT;
  size_t dnu, inv_dnu, two_nu, nu_c, edges;
  size_t geo, xe, ye, nodes;
  size_t wx, wy, binpart, active;   // active bins: volume weights, partial sums, flags
  size_t kabs, kflux, jsrc;         // band grids: per band and cell tables
  size_t partial, result;
  size_t total;
};

constexpr int kResBlocks = 1024;
constexpr int kMaxActiveBins = 8192;    // the selection keeps W_k in LDS (64 KB)
constexpr int kDynRslBlocks = 1024;     // block maxima of m1_dynamic_c_tilde (8 KiB of d_work)
constexpr double kEpsRsl = 4.0;         // Section 2.1 defaults of the dynamic
constexpr double kCTildeMin = 1.0e7;    // reduced speed of light (100 km/s)

// Device bytes the set-up needs for temporaries: the input fields (when they
// come from the host), class sums and tables, face velocities in double.
size_t init_temp_need(size_t nc, int nb, int64_t ncls, int nx, int ny, bool host_fields) {
  size_t need = host_fields ? 8 * align_up(nc * sizeof(double)) : 0;
  need += 2 * align_up(ncls * sizeof(double)) + align_up((size_t)ncls * nb * sizeof(double));
  need += 2 * ((size_t)(nx + 1) * ny + (size_t)nx * (ny + 1)) * sizeof(double);
  return need;
}

Layout make_layout(int nx, int ny, int nb, int64_t ncls, size_t rs) {
  Layout L{};
  size_t off = 0;
  size_t nc = (size_t)nx * ny, nbc = (size_t)nb * nc;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
  for (int b = 0; b < 2; ++b)
    for (int f = 0; f < 3; ++f) L.state[b][f] = take(nbc * rs);
  L.zw = take(2 * nbc * rs);
  // the set-up borrows the second state buffer and the scratch; with few
  // bins that span is padded up to the set-up's need
  const size_t span = off - L.state[1][0];
  const size_t need = init_temp_need(nc, nb, ncls > 0 ? ncls : (int64_t)nc, nx, ny, true);
  if (span < need) take(need - span);
  L.force = take(4 * nc * sizeof(double));
  L.cls = take(nc * sizeof(int32_t));
  L.island = take(nc);
  L.alpha = take(nc * rs);
  L.acF = take(nc * rs);
  L.acabs = take(nc * rs);
  L.pda = take(nc * rs);
  L.em = take(nc * rs);
  L.grad = take(4 * nc * rs);
  L.ufx = take((size_t)(nx + 1) * ny * rs);
  L.ufy = take((size_t)nx * (ny + 1) * rs);
  L.hbar = take((size_t)ncls * nb * rs);
  L.phi = take((size_t)ncls * nb * rs);
  L.dD2h = take((size_t)ncls * sizeof(double));
  L.hkT = take((size_t)ncls * sizeof(double));
  L.dnu = take(nb * sizeof(double));
  L.inv_dnu = take(nb * sizeof(double));
  L.two_nu = take(nb * sizeof(double));
  L.nu_c = take(nb * sizeof(double));
  L.edges = take((nb + 1) * sizeof(double));
  L.geo = take((size_t)(3 * (nx + 4) + 3 * nx + 3 * (ny + 4) + ny) * rs);
  L.xe = take((nx + 1) * sizeof(double));
  L.ye = take((ny + 1) * sizeof(double));
  L.wx = take(nx * sizeof(double));
  L.wy = take(ny * sizeof(double));
  L.binpart = take((size_t)nb * energy_chunks(nc) * sizeof(double));
  L.active = take(nb * sizeof(int32_t));
  L.nodes = take(kDawsonNodes * sizeof(double));
  L.partial = take(3 * kResBlocks * sizeof(double));
  L.result = take(2 * sizeof(double));
  L.total = off;
  return L;
}

constexpr int kMaxBands = 1024;

// Device bytes the band set-up needs for temporaries: the velocities (when
// they come from the host) and the face velocities in double.
size_t band_temp_need(size_t nc, int nx, int ny, bool host_fields) {
  size_t need = host_fields ? 2 * align_up(nc * sizeof(double)) : 0;
  return need + 2 * ((size_t)(nx + 1) * ny + (size_t)nx * (ny + 1)) * sizeof(double);
}

// Workspace of a grid of nb broad bands: state, per band and cell tables,
// velocity data, geometry, force and the residual's partial sums.
Layout make_band_layout(int nx, int ny, int nb, size_t rs) {
  Layout L{};
  size_t off = 0;
  size_t nc = (size_t)nx * ny, nbc = (size_t)nb * nc;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
  for (int b = 0; b < 2; ++b)
    for (int f = 0; f < 3; ++f) L.state[b][f] = take(nbc * rs);
  // the set-up borrows the second state buffer, padded up to its need
  const size_t span = off - L.state[1][0];
  const size_t need = band_temp_need(nc, nx, ny, true);
  if (span < need) take(need - span);
  L.force = take(4 * nc * sizeof(double));
  L.kabs = take(nbc * rs);
  L.kflux = take(nbc * rs);
  L.jsrc = take(nbc * rs);
  L.grad = take(4 * nc * rs);
  L.ufx = take((size_t)(nx + 1) * ny * rs);
  L.ufy = take((size_t)nx * (ny + 1) * rs);
  L.geo = take((size_t)(3 * (nx + 4) + 3 * nx + 3 * (ny + 4) + ny) * rs);
  L.xe = take((nx + 1) * sizeof(double));
  L.ye = take((ny + 1) * sizeof(double));
  L.partial = take(3 * kResBlocks * sizeof(double));
  L.result = take(2 * sizeof(double));
  L.total = off;
  return L;
}

int validate_config(const m1_config* c, int* nb_out) {
  if (!c) return fail(M1_EINVAL, "config is NULL");
  if (c->geom != M1_CART2D && c->geom != M1_CYL_RZ) return fail(M1_EINVAL, "bad geom %d", c->geom);
  if (c->nx < 4 || c->ny < 4) return fail(M1_EINVAL, "nx, ny must be >= 4");
  if ((int64_t)c->nx * c->ny > ((int64_t)1 << 31)) return fail(M1_EINVAL, "grid too large");
  if (!(c->x1 > c->x0) || !(c->y1 > c->y0) || !isfinite(c->x0) || !isfinite(c->x1) ||
      !isfinite(c->y0) || !isfinite(c->y1))
    return fail(M1_EINVAL, "bad domain edges");
  for (int s = 0; s < 4; ++s)
    if (c->bc[s] != M1_BC_VACUUM && c->bc[s] != M1_BC_REFLECT)
      return fail(M1_EINVAL, "bad boundary code on side %d", s);
  if (c->geom == M1_CYL_RZ && (c->x0 != 0.0 || c->bc[0] != M1_BC_REFLECT))
    return fail(M1_EINVAL, "cylindrical grids start on the axis (x0 = 0, reflecting x-)");
  if (!(c->c_tilde > 0.0) || c->c_tilde > kC) return fail(M1_EINVAL, "need 0 < c_tilde <= c");
  if (!(c->cfl > 0.0) || c->cfl > 1.0) return fail(M1_EINVAL, "need 0 < cfl <= 1");
  if (c->prec != M1_FP64 && c->prec != M1_FP32) return fail(M1_EINVAL, "bad precision");
  if (c->recoil != 0 && c->recoil != 1) return fail(M1_EINVAL, "recoil must be 0/1");
  if (c->doppler != 0 && c->doppler != 1) return fail(M1_EINVAL, "doppler must be 0/1");
  if ((int64_t)c->nx * c->ny > (int64_t(1) << 29))
    return fail(M1_EUNSUPPORTED, "more than 2^29 cells in one grid");
  if (isnan(c->fp64_tau)) return fail(M1_EINVAL, "fp64_tau is NaN");
  if (!(c->active_frac >= 0.0) || !isfinite(c->active_frac))
    return fail(M1_EINVAL, "active_frac must be finite and >= 0");
  if (c->substep_rule != 0 && c->substep_rule != 1) return fail(M1_EINVAL, "substep_rule must be 0/1");
  if (c->flux != M1_FLUX_GLF && c->flux != M1_FLUX_HLL_EIG) return fail(M1_EINVAL, "bad flux %d", c->flux);
  if (c->flux == M1_FLUX_HLL_EIG && (c->active_frac != 0.0 || c->substep_rule))
    return fail(M1_EUNSUPPORTED, "the eigenvalue HLL flux takes neither active bins nor substeps");
  FreqGrid g;
  int st = build_grid(*c, g);
  if (st) return st;
  if (c->active_frac > 0.0 && g.nb > kMaxActiveBins)
    return fail(M1_EUNSUPPORTED, "active-bin selection supports at most %d bins", kMaxActiveBins);
  if (nb_out) *nb_out = g.nb;
  return M1_OK;
}

}  // namespace

struct m1_handle {
  m1_config cfg;
  int nb = 0;
  int64_t ncls = 0;
  size_t nc = 0;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  Layout L;
  double dt = 0.0;
  int e2 = 0;                 // internal state = physical state * 2^e2
  int cur = 0;                // state buffer holding the current state
  int64_t steps = 0;
  double t = 0.0;
  GridArgs<float> af[2];
  GridArgs<double> ad[2];
  bool broken = false;
  bool band = false;          // a grid of broad bands (m1_band_init)
  double umax = 0.0;          // largest gas speed (the CFL step's |u|)
  int64_t gen = 0;            // bumped when the kernel arguments change
};

namespace {

template <typename R>
void fill_args(m1_handle* h, GridArgs<R>* a) {
  const m1_config& c = h->cfg;
  const Layout& L = h->L;
  char* w = h->ws;
  int nx = c.nx, ny = c.ny;
  for (int dir = 0; dir < 2; ++dir) {
    GridArgs<R>& g = a[dir];
    g.nx = nx; g.ny = ny; g.nb = h->nb; g.geom = c.geom;
    for (int s = 0; s < 4; ++s) g.bc[s] = c.bc[s];
    g.recoil = c.recoil; g.doppler = c.doppler;
    g.islands = (c.prec == M1_FP32 && c.fp64_tau < INFINITY) ? 1 : 0;
    g.ctdt = (R)(c.c_tilde * h->dt);
    g.ctdt_c = (R)(c.c_tilde * h->dt / kC);
    int in = dir, out = dir ^ 1;
    g.E = (const R*)(w + L.state[in][0]);
    g.fx = (const R*)(w + L.state[in][1]);
    g.fy = (const R*)(w + L.state[in][2]);
    g.Eo = (R*)(w + L.state[out][0]);
    g.fxo = (R*)(w + L.state[out][1]);
    g.fyo = (R*)(w + L.state[out][2]);
    g.cls = (const int32_t*)(w + L.cls);
    g.island = (const uint8_t*)(w + L.island);
    g.alpha = (const R*)(w + L.alpha);
    g.acF = (const R*)(w + L.acF);
    g.acabs = (const R*)(w + L.acabs);
    g.pda = (const R*)(w + L.pda);
    g.em = (const R*)(w + L.em);
    g.grad = (const R*)(w + L.grad);
    g.ufx = (const R*)(w + L.ufx);
    g.ufy = (const R*)(w + L.ufy);
    g.hbar = (const R*)(w + L.hbar);
    g.phi = (const R*)(w + L.phi);
    g.dD2h = (const double*)(w + L.dD2h);
    g.hkT = (const double*)(w + L.hkT);
    g.dnu = (const double*)(w + L.dnu);
    g.inv_dnu = (const double*)(w + L.inv_dnu);
    g.two_nu = (const double*)(w + L.two_nu);
    g.nu_c = (const double*)(w + L.nu_c);
    const R* geo = (const R*)(w + L.geo);
    g.xidl = geo;
    g.xhm = geo + (nx + 4);
    g.xhp = geo + 2 * (nx + 4);
    g.cxm = geo + 3 * (nx + 4);
    g.cxp = g.cxm + nx;
    g.chp = g.cxp + nx;
    g.yidl = g.chp + nx;
    g.yhm = g.yidl + (ny + 4);
    g.yhp = g.yhm + (ny + 4);
    g.cy = g.yhp + (ny + 4);
    g.zw = (ZW<R>*)(w + L.zw);
    g.force = (double*)(w + L.force);
    g.active = c.active_frac > 0.0 ? (const int32_t*)(w + L.active) : nullptr;
    g.substeps = c.substep_rule;
    g.flux = c.flux;
    g.kabs = g.kflux = g.jsrc = nullptr;
    // e_floor = 4 pi J_floor / c, J_floor = 1e-15 erg cm^-2 s^-1 sr^-1, in
    // the scaled state units
    g.e_floor = ldexp(4.0 * kPi * 1.0e-15 / kC, h->e2);
  }
}

// Cell centroids including two ghost layers, and the derived geometric
// factors of the reconstruction and the conservative update.
template <typename R>
std::vector<R> build_geometry(const m1_config& c, double ctdt, std::vector<double>& xe,
                              std::vector<double>& ye) {
  int nx = c.nx, ny = c.ny;
  bool cyl = c.geom == M1_CYL_RZ;
  xe.resize(nx + 1);
  ye.resize(ny + 1);
  for (int i = 0; i <= nx; ++i) xe[i] = c.x0 + (c.x1 - c.x0) * i / nx;
  for (int j = 0; j <= ny; ++j) ye[j] = c.y0 + (c.y1 - c.y0) * j / ny;
  auto centR = [](double a, double b) { return (2.0 / 3.0) * (b * b * b - a * a * a) / (b * b - a * a); };
  // centroids, index i + 2 for i in [-2, nx+1]
  std::vector<double> xc(nx + 4), yc(ny + 4);
  for (int i = 0; i < nx; ++i) xc[i + 2] = cyl ? centR(xe[i], xe[i + 1]) : 0.5 * (xe[i] + xe[i + 1]);
  for (int j = 0; j < ny; ++j) yc[j + 2] = 0.5 * (ye[j] + ye[j + 1]);
  double dxl = xe[1] - xe[0], dxr = xe[nx] - xe[nx - 1];
  double dyl = ye[1] - ye[0], dyr = ye[ny] - ye[ny - 1];
  for (int g = 1; g <= 2; ++g) {
    if (c.bc[0] == M1_BC_REFLECT) xc[2 - g] = 2.0 * xe[0] - xc[1 + g];
    else { double a = xe[0] - g * dxl, b = a + dxl; xc[2 - g] = cyl ? centR(a, b) : 0.5 * (a + b); }
    if (c.bc[1] == M1_BC_REFLECT) xc[nx + 1 + g] = 2.0 * xe[nx] - xc[nx + 2 - g];
    else { double a = xe[nx] + (g - 1) * dxr, b = a + dxr; xc[nx + 1 + g] = cyl ? centR(a, b) : 0.5 * (a + b); }
    if (c.bc[2] == M1_BC_REFLECT) yc[2 - g] = 2.0 * ye[0] - yc[1 + g];
    else yc[2 - g] = ye[0] - (g - 0.5) * dyl;
    if (c.bc[3] == M1_BC_REFLECT) yc[ny + 1 + g] = 2.0 * ye[ny] - yc[ny + 2 - g];
    else yc[ny + 1 + g] = ye[ny] + (g - 0.5) * dyr;
  }
  std::vector<R> geo(3 * (nx + 4) + 3 * nx + 3 * (ny + 4) + ny, R(0));
  R* xidl = geo.data();
  R* xhm = xidl + (nx + 4);
  R* xhp = xhm + (nx + 4);
  R* cxm = xhp + (nx + 4);
  R* cxp = cxm + nx;
  R* chp = cxp + nx;
  R* yidl = chp + nx;
  R* yhm = yidl + (ny + 4);
  R* yhp = yhm + (ny + 4);
  R* cy = yhp + (ny + 4);
  auto xedge = [&](int i) { return i < 0 ? xe[0] + i * dxl : (i > nx ? xe[nx] + (i - nx) * dxr : xe[i]); };
  auto yedge = [&](int j) { return j < 0 ? ye[0] + j * dyl : (j > ny ? ye[ny] + (j - ny) * dyr : ye[j]); };
  for (int i = -1; i <= nx + 1; ++i) xidl[i + 2] = (R)(1.0 / (xc[i + 2] - xc[i + 1]));
  for (int i = -1; i <= nx; ++i) {
    xhm[i + 2] = (R)(xedge(i) - xc[i + 2]);
    xhp[i + 2] = (R)(xedge(i + 1) - xc[i + 2]);
  }
  for (int i = 0; i < nx; ++i) {
    double a = xe[i], b = xe[i + 1];
    if (cyl) {
      double den = b * b - a * a;
      cxm[i] = (R)(ctdt * 2.0 * a / den);
      cxp[i] = (R)(ctdt * 2.0 * b / den);
      chp[i] = (R)(ctdt * 2.0 * (b - a) / den);
    } else {
      cxm[i] = cxp[i] = (R)(ctdt / (b - a));
      chp[i] = R(0);
    }
  }
  for (int j = -1; j <= ny + 1; ++j) yidl[j + 2] = (R)(1.0 / (yc[j + 2] - yc[j + 1]));
  for (int j = -1; j <= ny; ++j) {
    yhm[j + 2] = (R)(yedge(j) - yc[j + 2]);
    yhp[j + 2] = (R)(yedge(j + 1) - yc[j + 2]);
  }
  for (int j = 0; j < ny; ++j) cy[j] = (R)(ctdt / (ye[j + 1] - ye[j]));
  return geo;
}

int count_classes(const double* T, size_t n, std::vector<int32_t>* cls, std::vector<double>* vals) {
  std::unordered_map<uint64_t, int32_t> m;
  m.reserve(64);
  if (cls) cls->resize(n);
  for (size_t c = 0; c < n; ++c) {
    uint64_t bits;
    memcpy(&bits, &T[c], 8);
    auto it = m.find(bits);
    int32_t id;
    if (it == m.end()) {
      id = (int32_t)m.size();
      m.emplace(bits, id);
      if (vals) vals->push_back(T[c]);
    } else {
      id = it->second;
    }
    if (cls) (*cls)[c] = id;
  }
  return (int)m.size();
}

template <typename R>
int init_typed(m1_handle* h, const m1_fields* f, const std::vector<std::vector<double>>& host,
               const FreqGrid& g, const std::vector<int32_t>& cls,
               const std::vector<double>& Tcls) {
  const m1_config& c = h->cfg;
  hipStream_t s = h->stream;
  char* w = h->ws;
  const Layout& L = h->L;
  size_t nc = h->nc;
  int nb = g.nb;
  int nx = c.nx, ny = c.ny;
  // temporary area for set-up: second state buffer + frequency scratch
  char* tmp = w + L.state[1][0];
  // (spans state buffer 1 and the two frequency-step scratch arrays only)
  // inputs on the device
  CellInputs in;
  const double* dev[8];
  if (f->on_device) {
    const double* p[8] = {f->n_HI, f->T, f->u_x, f->u_y, f->alpha_abs, f->alpha_flux, f->p_d, f->emis};
    for (int q = 0; q < 8; ++q) dev[q] = p[q];
  } else {
    for (int q = 0; q < 8; ++q) {
      double* d = (double*)(tmp + (size_t)q * align_up(nc * sizeof(double)));
      HIPCHK(hipMemcpyAsync(d, host[q].data(), nc * sizeof(double), hipMemcpyHostToDevice, s));
      dev[q] = d;
    }
  }
  char* tmp2 = tmp + (f->on_device ? 0 : 8 * align_up(nc * sizeof(double)));
  in.n_HI = dev[0]; in.T = dev[1]; in.ux = dev[2]; in.uy = dev[3];
  in.acabs = dev[4]; in.acF = dev[5]; in.pd = dev[6]; in.emis = dev[7];

  // CFL time step and state scale from device reductions
  int nblk = (int)std::min<size_t>((nc + 255) / 256, kResBlocks);
  double* part = (double*)(w + L.partial);
  HIPCHK(launch_init_reduce(in, nc, part, nblk, s));
  std::vector<double> hp(3 * nblk);
  HIPCHK(hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  double umax = 0, emax = 0, tmin = 1e300;
  for (int b = 0; b < nblk; ++b) {
    umax = std::max(umax, hp[3 * b]);
    emax = std::max(emax, hp[3 * b + 1]);
    tmin = std::min(tmin, hp[3 * b + 2]);
  }
  double dx = (c.x1 - c.x0) / c.nx, dy = (c.y1 - c.y0) / c.ny;
  double dmin = std::min(dx, dy);
  h->dt = c.cfl * 0.5 * (dmin / (c.c_tilde + umax));
  h->umax = umax;
  double ctdt = c.c_tilde * h->dt;
  // internal scale: first-step line-centre energy density of the brightest
  // cell ~ 1 (exact power of two, so results are scaled exactly)
  double v = ctdt * emax / (kC * kSqrtPi * doppler_width(tmin));
  int e2 = 0;
  if (v > 0 && isfinite(v)) e2 = -(int)floor(log2(v));
  e2 = std::max(-900, std::min(900, e2));
  h->e2 = e2;

  // per-bin constants, classes, Dawson nodes, geometry
  std::vector<double> two_nu(nb), nu_c(nb), inv_dnu(nb);
  for (int k = 0; k < nb; ++k) {
    two_nu[k] = 2.0 / g.nuc[k];
    nu_c[k] = g.nuc[k] / kC;
    inv_dnu[k] = 1.0 / g.dnu[k];
  }
  HIPCHK(hipMemcpyAsync(w + L.inv_dnu, inv_dnu.data(), nb * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(w + L.dnu, g.dnu.data(), nb * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(w + L.two_nu, two_nu.data(), nb * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(w + L.nu_c, nu_c.data(), nb * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(w + L.edges, g.edges.data(), (nb + 1) * sizeof(double), hipMemcpyHostToDevice, s));
  std::vector<double> nodes(kDawsonNodes);
  dawson_nodes_host(nodes.data());
  HIPCHK(hipMemcpyAsync(w + L.nodes, nodes.data(), kDawsonNodes * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(w + L.cls, cls.data(), nc * sizeof(int32_t), hipMemcpyHostToDevice, s));
  int64_t ncls = (int64_t)Tcls.size();
  std::vector<double> dD2h(ncls), hkT(ncls), dD(ncls), av(ncls);
  for (int64_t q = 0; q < ncls; ++q) {
    double T = Tcls[q];
    dD[q] = doppler_width(T);
    dD2h[q] = 0.5 * dD[q] * dD[q];
    hkT[q] = kHP / (kKB * T);
    av[q] = 4.7e-4 / sqrt(T / 1.0e4);
  }
  HIPCHK(hipMemcpyAsync(w + L.dD2h, dD2h.data(), ncls * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(w + L.hkT, hkT.data(), ncls * sizeof(double), hipMemcpyHostToDevice, s));
  double* d_dD = (double*)tmp2;
  double* d_av = (double*)(tmp2 + align_up(ncls * sizeof(double)));
  double* d_htmp = (double*)(tmp2 + 2 * align_up(ncls * sizeof(double)));
  HIPCHK(hipMemcpyAsync(d_dD, dD.data(), ncls * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(d_av, av.data(), ncls * sizeof(double), hipMemcpyHostToDevice, s));
  std::vector<double> xe, ye;
  std::vector<R> geo = build_geometry<R>(c, ctdt, xe, ye);
  HIPCHK(hipMemcpyAsync(w + L.geo, geo.data(), geo.size() * sizeof(R), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(w + L.xe, xe.data(), xe.size() * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(w + L.ye, ye.data(), ye.size() * sizeof(double), hipMemcpyHostToDevice, s));
  // cell volumes dV = wx[i] wy[j] (cylindrical: pi (R+^2 - R-^2) dz; slab:
  // unit depth) for the active-bin energies; no bin is flagged before a step
  std::vector<double> wxv(nx), wyv(ny);
  for (int i = 0; i < nx; ++i)
    wxv[i] = c.geom == M1_CYL_RZ ? kPi * (xe[i + 1] * xe[i + 1] - xe[i] * xe[i]) : xe[i + 1] - xe[i];
  for (int j = 0; j < ny; ++j) wyv[j] = ye[j + 1] - ye[j];
  HIPCHK(hipMemcpyAsync(w + L.wx, wxv.data(), nx * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(w + L.wy, wyv.data(), ny * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemsetAsync(w + L.active, 0, nb * sizeof(int32_t), s));

  // bin-averaged Voigt profile and emission profile per class
  HIPCHK(launch_class_profiles<R>(d_dD, d_av, ncls, (const double*)(w + L.edges),
                                  (const double*)(w + L.dnu), nb, (const double*)(w + L.nodes),
                                  d_htmp, (R*)(w + L.hbar), (R*)(w + L.phi), s));
  // per-cell opacities and emission
  HIPCHK(launch_cell_setup<R>(in, nc, dmin, c.fp64_tau, e2, (R*)(w + L.alpha), (R*)(w + L.acF),
                              (R*)(w + L.acabs), (R*)(w + L.pda), (R*)(w + L.em),
                              (uint8_t*)(w + L.island), s));
  // velocity gradients and face velocities (face temp after the class temp)
  double* vtmp = (double*)(tmp2 + 2 * align_up(ncls * sizeof(double)) +
                           align_up((size_t)ncls * nb * sizeof(double)));
  HIPCHK(launch_velocity<R>(in, nx, ny, c.geom, c.bc, (const double*)(w + L.xe),
                            (const double*)(w + L.ye), vtmp, (R*)(w + L.ufx), (R*)(w + L.ufy),
                            (R*)(w + L.grad), s));
  HIPCHK(hipStreamSynchronize(s));
  // E = F = 0 in both buffers, force = 0
  for (int b = 0; b < 2; ++b)
    for (int q = 0; q < 3; ++q)
      HIPCHK(hipMemsetAsync(w + L.state[b][q], 0, (size_t)nb * nc * sizeof(R), s));
  HIPCHK(hipMemsetAsync(w + L.force, 0, 4 * nc * sizeof(double), s));
  HIPCHK(hipStreamSynchronize(s));
  return M1_OK;
}

// Kernel arguments of a band grid: state, band tables, velocity data,
// geometry and force; the line data stay null.
template <typename R>
void fill_band_args(m1_handle* h, GridArgs<R>* a) {
  const m1_config& c = h->cfg;
  const Layout& L = h->L;
  char* w = h->ws;
  const int nx = c.nx, ny = c.ny;
  for (int dir = 0; dir < 2; ++dir) {
    GridArgs<R> g{};
    g.nx = nx; g.ny = ny; g.nb = h->nb; g.geom = c.geom;
    for (int q = 0; q < 4; ++q) g.bc[q] = c.bc[q];
    g.ctdt = (R)(c.c_tilde * h->dt);
    g.ctdt_c = (R)(c.c_tilde * h->dt / kC);
    const int in = dir, out = dir ^ 1;
    g.E = (const R*)(w + L.state[in][0]);
    g.fx = (const R*)(w + L.state[in][1]);
    g.fy = (const R*)(w + L.state[in][2]);
    g.Eo = (R*)(w + L.state[out][0]);
    g.fxo = (R*)(w + L.state[out][1]);
    g.fyo = (R*)(w + L.state[out][2]);
    g.grad = (const R*)(w + L.grad);
    g.ufx = (const R*)(w + L.ufx);
    g.ufy = (const R*)(w + L.ufy);
    const R* geo = (const R*)(w + L.geo);
    g.xidl = geo;
    g.xhm = geo + (nx + 4);
    g.xhp = geo + 2 * (nx + 4);
    g.cxm = geo + 3 * (nx + 4);
    g.cxp = g.cxm + nx;
    g.chp = g.cxp + nx;
    g.yidl = g.chp + nx;
    g.yhm = g.yidl + (ny + 4);
    g.yhp = g.yhm + (ny + 4);
    g.cy = g.yhp + (ny + 4);
    g.force = (double*)(w + L.force);
    g.kabs = (const R*)(w + L.kabs);
    g.kflux = (const R*)(w + L.kflux);
    g.jsrc = (const R*)(w + L.jsrc);
    a[dir] = g;
  }
}

// Band set-up: tables in the state precision (emission as 2^e2 L / c), face
// velocities and gradients, geometry, zero state and force.  host: the
// validated inputs (u_x, u_y, kappa_abs, kappa_flux, emis).
template <typename R>
int band_init_typed(m1_handle* h, const m1_band_fields* f,
                    const std::vector<std::vector<double>>& host, double umax, double jmax) {
  const m1_config& c = h->cfg;
  hipStream_t s = h->stream;
  char* w = h->ws;
  const Layout& L = h->L;
  const size_t nc = h->nc, nbc = (size_t)h->nb * nc;
  const int nx = c.nx, ny = c.ny;
  const double dx = (c.x1 - c.x0) / nx, dy = (c.y1 - c.y0) / ny;
  h->dt = c.cfl * 0.5 * (std::min(dx, dy) / (c.c_tilde + umax));
  h->umax = umax;
  const double ctdt = c.c_tilde * h->dt;
  // internal scale: the brightest cell's first-step emission ~ 1 (a power
  // of two, so results are scaled exactly)
  const double v = ctdt * jmax / kC;
  int e2 = 0;
  if (v > 0 && isfinite(v)) e2 = -(int)floor(log2(v));
  h->e2 = std::max(-900, std::min(900, e2));
  std::vector<R> t(nbc);
  const size_t off[3] = {L.kabs, L.kflux, L.jsrc};
  for (int q = 0; q < 3; ++q) {
    const std::vector<double>& src = host[2 + q];
    for (size_t i = 0; i < nbc; ++i) t[i] = (R)(q == 2 ? ldexp(src[i], h->e2) / kC : src[i]);
    HIPCHK(hipMemcpyAsync(w + off[q], t.data(), nbc * sizeof(R), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));          // t is reused
  }
  std::vector<double> xe, ye;
  std::vector<R> geo = build_geometry<R>(c, ctdt, xe, ye);
  HIPCHK(hipMemcpyAsync(w + L.geo, geo.data(), geo.size() * sizeof(R), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(w + L.xe, xe.data(), xe.size() * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(w + L.ye, ye.data(), ye.size() * sizeof(double), hipMemcpyHostToDevice, s));
  // velocities: the caller's device arrays, or copies in the borrowed
  // second state buffer; the face-velocity temporaries after them
  char* tmp = w + L.state[1][0];
  CellInputs in{};
  if (f->on_device) {
    in.ux = f->u_x;
    in.uy = f->u_y;
  } else {
    double* ux = (double*)tmp;
    double* uy = (double*)(tmp + align_up(nc * sizeof(double)));
    HIPCHK(hipMemcpyAsync(ux, host[0].data(), nc * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(uy, host[1].data(), nc * sizeof(double), hipMemcpyHostToDevice, s));
    in.ux = ux;
    in.uy = uy;
    tmp += 2 * align_up(nc * sizeof(double));
  }
  HIPCHK(launch_velocity<R>(in, nx, ny, c.geom, c.bc, (const double*)(w + L.xe),
                            (const double*)(w + L.ye), (double*)tmp, (R*)(w + L.ufx),
                            (R*)(w + L.ufy), (R*)(w + L.grad), s));
  HIPCHK(hipStreamSynchronize(s));
  for (int b = 0; b < 2; ++b)
    for (int q = 0; q < 3; ++q) HIPCHK(hipMemsetAsync(w + L.state[b][q], 0, nbc * sizeof(R), s));
  HIPCHK(hipMemsetAsync(w + L.force, 0, 4 * nc * sizeof(double), s));
  HIPCHK(hipStreamSynchronize(s));
  return M1_OK;
}

}  // namespace

// =========================================================================
namespace m1 {
int record_error(int code, const char* msg) {
  g_err = msg;
  return code;
}
}  // namespace m1

// ---- scratch of the entry point without allocation.  A file-scope device
// array (one copy per GPU, alive until the process ends): the block maxima
// of the dynamic reduced speed of light and, after them, their maximum.  In
// host code `scratch` names a host-side stand-in, never a device address:
// kernels and copies use the per-device address from hipGetSymbolAddress.
constexpr int kScratchDoubles = kDynRslBlocks + 32;           // 8448 bytes
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

// Arguments of the dynamic reduced speed of light, checked before any
// device work: cell inputs, cell count and the larger cell side.
int dyn_rsl_args(const m1_config* cfg, const m1_fields* f, const double* d_cs, double c_prev,
                 double* c_tilde, CellInputs* in, size_t* nc, double* dmax) {
  int st = validate_config(cfg, nullptr);
  if (st) return st;
  if (!f || !d_cs || !c_tilde) return fail(M1_EINVAL, "NULL argument");
  if (!f->on_device) return fail(M1_EINVAL, "fields must be device arrays (on_device = 1)");
  if (!f->n_HI || !f->T || !f->u_x || !f->u_y || !f->alpha_abs || !f->p_d)
    return fail(M1_EINVAL, "a field array is NULL");
  if (!(c_prev >= 0.0) || !isfinite(c_prev)) return fail(M1_EINVAL, "c_prev must be finite and >= 0");
  *nc = (size_t)cfg->nx * cfg->ny;
  *dmax = std::max((cfg->x1 - cfg->x0) / cfg->nx, (cfg->y1 - cfg->y0) / cfg->ny);
  *in = CellInputs{f->n_HI, f->T, f->u_x, f->u_y, f->alpha_abs, f->alpha_flux, f->p_d, f->emis};
  return M1_OK;
}

// c_tilde = min(max(c_min, eps_RSL m), c), rate-limited against c_prev > 0.
int dyn_rsl_finish(double m, double c_prev, double* c_tilde) {
  if (m != m) return fail(M1_EINVAL, "non-finite trapping term (check T > 0 and the opacities)");
  double c = std::min(std::max(kCTildeMin, kEpsRsl * m), kC);
  if (c_prev > 0.0) c = std::min(std::max(c, 0.75 * c_prev), 4.0 * c_prev);
  *c_tilde = c;
  return M1_OK;
}

// Devices whose scratch address is kept.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_dev[kMaxDevices] = {};

// Device address of the current device's scratch, looked up once per device
// (the first call on that device, with the device current).
int scratch_address(double** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(M1_EDEVICE, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(M1_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_dev[dev] = (double*)p;
  }
  *out = g_scratch_dev[dev];
  return M1_OK;
}

}  // namespace

extern "C" {

const char* m1_last_error(void) { return g_err.c_str(); }

int32_t m1_default_config(m1_config* c) {
  if (!c) return fail(M1_EINVAL, "config is NULL");
  memset(c, 0, sizeof *c);
  c->geom = M1_CART2D;
  c->nx = c->ny = 64;
  c->x0 = 0; c->x1 = 1; c->y0 = 0; c->y1 = 1;
  for (int s = 0; s < 4; ++s) c->bc[s] = M1_BC_VACUUM;
  c->T_min = 30.0;
  c->q = 1.1;
  c->half_width = 1.0e5;
  c->c_tilde = 0.01 * kC;
  c->cfl = 0.4;
  c->recoil = 1;
  c->doppler = 1;
  c->prec = M1_FP64;
  c->fp64_tau = INFINITY;
  return M1_OK;
}

int32_t m1_num_bins(const m1_config* cfg, int32_t* n_nu) {
  if (!n_nu) return fail(M1_EINVAL, "n_nu is NULL");
  int nb = 0;
  int st = validate_config(cfg, &nb);
  if (st) return st;
  *n_nu = nb;
  return M1_OK;
}

int32_t m1_frequency_grid(const m1_config* cfg, double* nu_centre, double* dnu) {
  int st = validate_config(cfg, nullptr);
  if (st) return st;
  FreqGrid g;
  st = build_grid(*cfg, g);
  if (st) return st;
  if (nu_centre) memcpy(nu_centre, g.nuc.data(), g.nb * sizeof(double));
  if (dnu) memcpy(dnu, g.dnu.data(), g.nb * sizeof(double));
  return M1_OK;
}


int32_t m1_dynamic_c_tilde(const m1_config* cfg, const m1_fields* f, const double* d_cs,
                           double c_prev, void* d_work, void* stream, double* c_tilde) {
  CellInputs in;
  size_t nc = 0;
  double dmax = 0.0;
  int st = dyn_rsl_args(cfg, f, d_cs, c_prev, c_tilde, &in, &nc, &dmax);
  if (st) return st;
  if (!d_work) return fail(M1_EINVAL, "NULL argument");
  if (((uintptr_t)d_work) & 7) return fail(M1_EINVAL, "d_work not 8-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  const int nblk = (int)std::min<size_t>((nc + 255) / 256, kDynRslBlocks);
  HIPCHK(launch_dyn_rsl(in, d_cs, nc, dmax, (double*)d_work, nblk, s));
  std::vector<double> part(nblk);
  HIPCHK(hipMemcpyAsync(part.data(), d_work, nblk * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  double m = 0.0;
  for (double v : part) {
    if (v != v) return dyn_rsl_finish(v, c_prev, c_tilde);
    m = std::max(m, v);
  }
  return dyn_rsl_finish(m, c_prev, c_tilde);
}

int32_t m1_dynamic_c_tilde_noalloc(const m1_config* cfg, const m1_fields* f,
                                   const double* d_cs, double c_prev, void* stream,
                                   double* c_tilde) {
  CellInputs in;
  size_t nc = 0;
  double dmax = 0.0;
  int st = dyn_rsl_args(cfg, f, d_cs, c_prev, c_tilde, &in, &nc, &dmax);
  if (st) return st;
  double* work = nullptr;
  st = scratch_address(&work);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  // every grid size fits: the kernel strides over the cells, so the block
  // maxima never outnumber kDynRslBlocks; the check states the bound
  const int nblk = (int)std::min<size_t>((nc + 255) / 256, kDynRslBlocks);
  if (nblk + 1 > kScratchDoubles)
    return fail(M1_EINVAL, "%d block maxima exceed the %d-double scratch", nblk, kScratchDoubles);
  HIPCHK(launch_dyn_rsl(in, d_cs, nc, dmax, work, nblk, s));
  HIPCHK(launch_max_of(work, nblk, work + kDynRslBlocks, s));
  double m = 0.0;
  HIPCHK(hipMemcpyAsync(&m, work + kDynRslBlocks, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return dyn_rsl_finish(m, c_prev, c_tilde);
}

int32_t m1_count_temperature_classes(const double* T, int64_t n, int64_t* n_classes) {
  if (!T || n <= 0 || !n_classes) return fail(M1_EINVAL, "bad arguments");
  *n_classes = count_classes(T, (size_t)n, nullptr, nullptr);
  return M1_OK;
}

int32_t m1_workspace_bytes(const m1_config* cfg, int64_t ncls, size_t* bytes) {
  if (!bytes) return fail(M1_EINVAL, "bytes is NULL");
  int nb = 0;
  int st = validate_config(cfg, &nb);
  if (st) return st;
  size_t nc = (size_t)cfg->nx * cfg->ny;
  if (ncls <= 0 || (size_t)ncls > nc) ncls = (int64_t)nc;
  size_t rs = cfg->prec == M1_FP32 ? 4 : 8;
  Layout L = make_layout(cfg->nx, cfg->ny, nb, ncls, rs);
  *bytes = L.total;
  return M1_OK;
}

int32_t m1_init(const m1_config* cfg, const m1_fields* f, void* d_ws, size_t ws_bytes,
                void* stream, m1_handle** out) {
  if (!out) return fail(M1_EINVAL, "out is NULL");
  *out = nullptr;
  int nb = 0;
  int st = validate_config(cfg, &nb);
  if (st) return st;
  if (!f) return fail(M1_EINVAL, "fields is NULL");
  const double* p[8] = {f->n_HI, f->T, f->u_x, f->u_y, f->alpha_abs, f->alpha_flux, f->p_d, f->emis};
  const char* names[8] = {"n_HI", "T", "u_x", "u_y", "alpha_abs", "alpha_flux", "p_d", "emis"};
  for (int q = 0; q < 8; ++q)
    if (!p[q]) return fail(M1_EINVAL, "field %s is NULL", names[q]);
  if (!d_ws) return fail(M1_EINVAL, "workspace is NULL");
  if (((uintptr_t)d_ws) & 255) return fail(M1_EINVAL, "workspace must be 256-byte aligned");
  size_t nc = (size_t)cfg->nx * cfg->ny;
  hipStream_t s = (hipStream_t)stream;
  // host view of the fields for validation and temperature classes
  std::vector<std::vector<double>> host(8);
  for (int q = 0; q < 8; ++q) {
    host[q].resize(nc);
    if (f->on_device) {
      HIPCHK(hipMemcpyAsync(host[q].data(), p[q], nc * sizeof(double), hipMemcpyDeviceToHost, s));
    } else {
      memcpy(host[q].data(), p[q], nc * sizeof(double));
    }
  }
  if (f->on_device) HIPCHK(hipStreamSynchronize(s));
  for (int q = 0; q < 8; ++q) {
    const std::vector<double>& v = host[q];
    bool signed_ok = (q == 2 || q == 3);
    for (size_t c = 0; c < nc; ++c) {
      if (!isfinite(v[c])) return fail(M1_EINVAL, "field %s has a non-finite value at %zu", names[q], c);
      if (!signed_ok && v[c] < 0) return fail(M1_EINVAL, "field %s is negative at %zu", names[q], c);
      if (q == 1 && !(v[c] > 0)) return fail(M1_EINVAL, "field T must be > 0 (cell %zu)", c);
      if (signed_ok && fabs(v[c]) >= kC) return fail(M1_EINVAL, "field %s reaches c at cell %zu", names[q], c);
    }
  }
  std::vector<int32_t> cls;
  std::vector<double> Tcls;
  count_classes(host[1].data(), nc, &cls, &Tcls);
  int64_t ncls = (int64_t)Tcls.size();
  size_t rs = cfg->prec == M1_FP32 ? 4 : 8;
  Layout L = make_layout(cfg->nx, cfg->ny, nb, ncls, rs);
  if (ws_bytes < L.total)
    return fail(M1_ENOMEM, "workspace of %zu bytes < %zu needed (%lld temperature classes)",
                ws_bytes, L.total, (long long)ncls);
  size_t tmp_cap = L.force - L.state[1][0];
  if (init_temp_need(nc, nb, ncls, cfg->nx, cfg->ny, !f->on_device) > tmp_cap)
    return fail(M1_EUNSUPPORTED, "set-up scratch does not fit the workspace layout");
  m1_handle* h = new m1_handle();
  h->cfg = *cfg;
  h->nb = nb;
  h->ncls = ncls;
  h->nc = nc;
  h->stream = s;
  h->ws = (char*)d_ws;
  h->L = L;
  FreqGrid g;
  build_grid(*cfg, g);
  if (cfg->prec == M1_FP32) st = init_typed<float>(h, f, host, g, cls, Tcls);
  else st = init_typed<double>(h, f, host, g, cls, Tcls);
  if (st) { delete h; return st; }
  fill_args<float>(h, h->af);
  fill_args<double>(h, h->ad);
  *out = h;
  return M1_OK;
}

int32_t m1_band_workspace_bytes(const m1_config* cfg, int32_t n_band, size_t* bytes) {
  if (!bytes) return fail(M1_EINVAL, "bytes is NULL");
  int st = validate_config(cfg, nullptr);
  if (st) return st;
  if (n_band < 1 || n_band > kMaxBands) return fail(M1_EINVAL, "need 1 <= n_band <= %d", kMaxBands);
  *bytes = make_band_layout(cfg->nx, cfg->ny, n_band, cfg->prec == M1_FP32 ? 4 : 8).total;
  return M1_OK;
}

int32_t m1_band_init(const m1_config* cfg, int32_t n_band, const m1_band_fields* f, void* d_ws,
                     size_t ws_bytes, void* stream, m1_handle** out) {
  if (!out) return fail(M1_EINVAL, "out is NULL");
  *out = nullptr;
  int st = validate_config(cfg, nullptr);
  if (st) return st;
  if (cfg->active_frac != 0.0 || cfg->substep_rule || cfg->flux != M1_FLUX_GLF)
    return fail(M1_EUNSUPPORTED,
                "band grids take neither active bins, the substep rule nor the eigenvalue HLL flux");
  if (n_band < 1 || n_band > kMaxBands) return fail(M1_EINVAL, "need 1 <= n_band <= %d", kMaxBands);
  if (!f) return fail(M1_EINVAL, "fields is NULL");
  const double* p[5] = {f->u_x, f->u_y, f->kappa_abs, f->kappa_flux, f->emis};
  const char* names[5] = {"u_x", "u_y", "kappa_abs", "kappa_flux", "emis"};
  for (int q = 0; q < 5; ++q)
    if (!p[q]) return fail(M1_EINVAL, "field %s is NULL", names[q]);
  if (!d_ws) return fail(M1_EINVAL, "workspace is NULL");
  if (((uintptr_t)d_ws) & 255) return fail(M1_EINVAL, "workspace must be 256-byte aligned");
  const size_t nc = (size_t)cfg->nx * cfg->ny, nbc = (size_t)n_band * nc;
  const size_t rs = cfg->prec == M1_FP32 ? 4 : 8;
  Layout L = make_band_layout(cfg->nx, cfg->ny, n_band, rs);
  if (ws_bytes < L.total)
    return fail(M1_ENOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, L.total);
  hipStream_t s = (hipStream_t)stream;
  std::vector<std::vector<double>> host(5);
  for (int q = 0; q < 5; ++q) {
    const size_t n = q < 2 ? nc : nbc;
    host[q].resize(n);
    if (f->on_device)
      HIPCHK(hipMemcpyAsync(host[q].data(), p[q], n * sizeof(double), hipMemcpyDeviceToHost, s));
    else
      memcpy(host[q].data(), p[q], n * sizeof(double));
  }
  if (f->on_device) HIPCHK(hipStreamSynchronize(s));
  double umax = 0.0, jmax = 0.0;
  for (int q = 0; q < 5; ++q) {
    const std::vector<double>& v = host[q];
    for (size_t i = 0; i < v.size(); ++i) {
      if (!isfinite(v[i])) return fail(M1_EINVAL, "field %s has a non-finite value at %zu", names[q], i);
      if (q >= 2 && v[i] < 0) return fail(M1_EINVAL, "field %s is negative at %zu", names[q], i);
      if (q < 2 && fabs(v[i]) >= kC) return fail(M1_EINVAL, "field %s reaches c at cell %zu", names[q], i);
      if (q == 4) jmax = std::max(jmax, v[i]);
    }
  }
  for (size_t i = 0; i < nc; ++i) umax = std::max(umax, hypot(host[0][i], host[1][i]));
  m1_handle* h = new m1_handle();
  h->cfg = *cfg;
  h->nb = n_band;
  h->ncls = 0;
  h->nc = nc;
  h->stream = s;
  h->ws = (char*)d_ws;
  h->L = L;
  h->band = true;
  st = cfg->prec == M1_FP32 ? band_init_typed<float>(h, f, host, umax, jmax)
                            : band_init_typed<double>(h, f, host, umax, jmax);
  if (st) { delete h; return st; }
  fill_band_args<float>(h, h->af);
  fill_band_args<double>(h, h->ad);
  *out = h;
  return M1_OK;
}

int32_t m1_active_bins(m1_handle* h, int32_t* flags_host, int32_t* n_active) {
  if (!h) return fail(M1_EINVAL, "handle is NULL");
  std::vector<int32_t> f(h->nb, 1);
  if (h->cfg.active_frac > 0.0) {
    HIPCHK(hipMemcpyAsync(f.data(), h->ws + h->L.active, h->nb * sizeof(int32_t),
                          hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
  }
  int32_t cnt = 0;
  for (int k = 0; k < h->nb; ++k) cnt += f[k] != 0;
  if (flags_host) memcpy(flags_host, f.data(), h->nb * sizeof(int32_t));
  if (n_active) *n_active = cnt;
  return M1_OK;
}

extern "C++" {
namespace {
template <typename R>
int set_geometry(m1_handle* h) {
  std::vector<double> xe, ye;
  std::vector<R> geo = build_geometry<R>(h->cfg, h->cfg.c_tilde * h->dt, xe, ye);
  HIPCHK(hipMemcpyAsync(h->ws + h->L.geo, geo.data(), geo.size() * sizeof(R),
                        hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return M1_OK;
}
}  // namespace
}  // extern "C++"

int32_t m1_set_c_tilde(m1_handle* h, double c_tilde) {
  if (!h) return fail(M1_EINVAL, "handle is NULL");
  if (h->broken) return fail(M1_ESTATE, "handle had a device error");
  if (!(c_tilde > 0.0) || !(c_tilde <= kC)) return fail(M1_EINVAL, "need 0 < c_tilde <= c");
  m1_config& c = h->cfg;
  c.c_tilde = c_tilde;
  const double dx = (c.x1 - c.x0) / c.nx, dy = (c.y1 - c.y0) / c.ny;
  h->dt = c.cfl * 0.5 * (std::min(dx, dy) / (c_tilde + h->umax));
  int st = c.prec == M1_FP32 ? set_geometry<float>(h) : set_geometry<double>(h);
  if (st) { h->broken = true; return st; }
  if (h->band) { fill_band_args<float>(h, h->af); fill_band_args<double>(h, h->ad); }
  else { fill_args<float>(h, h->af); fill_args<double>(h, h->ad); }
  h->gen += 1;
  return M1_OK;
}

int32_t m1_get_info(const m1_handle* h, double* dt, int32_t* n_nu, int32_t* prec, int64_t* ncell,
                    int32_t* scale_exp2) {
  if (!h) return fail(M1_EINVAL, "handle is NULL");
  if (dt) *dt = h->dt;
  if (n_nu) *n_nu = h->nb;
  if (prec) *prec = h->cfg.prec;
  if (ncell) *ncell = (int64_t)h->nc;
  if (scale_exp2) *scale_exp2 = h->e2;
  return M1_OK;
}

// Active-bin flags of the state in buffer `dir` (nothing when every bin is
// advected).
static hipError_t launch_selection(m1_handle* h, int dir, hipStream_t s) {
  if (!(h->cfg.active_frac > 0.0)) return hipSuccess;
  const Layout& L = h->L;
  char* w = h->ws;
  const double* wx = (const double*)(w + L.wx);
  const double* wy = (const double*)(w + L.wy);
  const double* dnu = (const double*)(w + L.dnu);
  double* part = (double*)(w + L.binpart);
  int32_t* act = (int32_t*)(w + L.active);
  const int nx = h->cfg.nx, ny = h->cfg.ny;
  return h->cfg.prec == M1_FP32
             ? launch_active_bins<float>((const float*)(w + L.state[dir][0]), nx, ny, h->nb, wx,
                                         wy, dnu, h->cfg.active_frac, part, act, s)
             : launch_active_bins<double>((const double*)(w + L.state[dir][0]), nx, ny, h->nb, wx,
                                          wy, dnu, h->cfg.active_frac, part, act, s);
}

static int enqueue_step(m1_handle* h, hipStream_t s) {
  hipError_t e = launch_selection(h, h->cur, s);
  if (e == hipSuccess && h->band)
    e = h->cfg.prec == M1_FP32 ? launch_band_step<float>(h->af[h->cur], s)
                               : launch_band_step<double>(h->ad[h->cur], s);
  else if (e == hipSuccess)
    e = h->cfg.prec == M1_FP32 ? launch_step<float>(h->af[h->cur], s)
                               : launch_step<double>(h->ad[h->cur], s);
  if (e != hipSuccess) {
    h->broken = true;
    return fail(M1_EDEVICE, "step launch failed: %s", hipGetErrorString(e));
  }
  h->cur ^= 1;
  h->steps += 1;
  h->t += h->dt;
  return M1_OK;
}

int32_t m1_step(m1_handle* h, int32_t nsteps, double* t_now) {
  if (!h) return fail(M1_EINVAL, "handle is NULL");
  if (h->broken) return fail(M1_ESTATE, "handle had a device error");
  if (nsteps < 0) return fail(M1_EINVAL, "nsteps < 0");
  for (int n = 0; n < nsteps; ++n) {
    int st = enqueue_step(h, h->stream);
    if (st) return st;
  }
  if (t_now) *t_now = h->t;
  return M1_OK;
}

int32_t m1_step_profiled(m1_handle* h, int32_t nsteps, double* ms) {
  if (!h || !ms) return fail(M1_EINVAL, "bad arguments");
  if (h->broken) return fail(M1_ESTATE, "handle had a device error");
  if (nsteps < 1 || nsteps > 4096) return fail(M1_EINVAL, "need 1 <= nsteps <= 4096");
  std::vector<hipEvent_t> ev(2 * nsteps + 1);
  for (auto& e : ev) HIPCHK(hipEventCreate(&e));
  int st = M1_OK;
  HIPCHK(hipEventRecord(ev[0], h->stream));
  for (int n = 0; n < nsteps && !st; ++n) {
    hipError_t e = launch_selection(h, h->cur, h->stream);
    if (e == hipSuccess && h->band)
      e = h->cfg.prec == M1_FP32 ? launch_band_step<float>(h->af[h->cur], h->stream)
                                 : launch_band_step<double>(h->ad[h->cur], h->stream);
    else if (e == hipSuccess)
      e = h->cfg.prec == M1_FP32 ? launch_advect<float>(h->af[h->cur], h->stream)
                                 : launch_advect<double>(h->ad[h->cur], h->stream);
    if (e == hipSuccess) e = hipEventRecord(ev[2 * n + 1], h->stream);
    if (e == hipSuccess && !h->band)
      e = h->cfg.prec == M1_FP32 ? launch_freq<float>(h->af[h->cur], h->stream)
                                 : launch_freq<double>(h->ad[h->cur], h->stream);
    if (e == hipSuccess) e = hipEventRecord(ev[2 * n + 2], h->stream);
    if (e != hipSuccess) { st = fail(M1_EDEVICE, "profiled step: %s", hipGetErrorString(e)); break; }
    h->cur ^= 1;
    h->steps += 1;
    h->t += h->dt;
  }
  if (!st) {
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) st = fail(M1_EDEVICE, "profiled step sync: %s", hipGetErrorString(e));
  }
  ms[0] = ms[1] = 0.0;
  for (int n = 0; n < nsteps && !st; ++n) {
    float a = 0, b = 0;
    (void)hipEventElapsedTime(&a, ev[2 * n], ev[2 * n + 1]);
    (void)hipEventElapsedTime(&b, ev[2 * n + 1], ev[2 * n + 2]);
    ms[0] += a;
    ms[1] += b;
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  return st;
}

}  // extern "C"

// ------------------------------------------------------------------ batches
struct m1_batch {
  std::vector<m1_handle*> hs;
  int n = 0;
  int prec = 0;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t args_off = 0, par_off = 0, offa_off = 0, offf_off = 0, offr_off = 0;
  std::vector<int> par;                 // base parity per grid
  int sp = 0;                           // steps taken mod 2
  int blocks_adv[kNumBatchVariants] = {};
  int blocks_freq = 0;
  int blocks_rates = 0;                 // rates items of the two-launch frequency step
  int islands = 0;                      // some member may have island cells
  int active = 0;                       // some member selects active bins
  bool fused_ok = false;                // the fused variant applies (float, no islands)
  int variant = -1;                     // chosen tile variant (-1: tuning)
  int trial_variant = 0, trial_step = 0;
  double trial_ms[kNumBatchVariants] = {};
  bool use_graph = false;
  hipGraphExec_t exec = nullptr;
  int graph_sp = -1;                    // parity at which the graph starts
  std::vector<int64_t> gen;             // members' argument generations uploaded
};

namespace {
constexpr int kTrialSteps = 2;          // timed steps per variant while tuning

size_t batch_layout(m1_handle* const* hs, int n, size_t* args_off, size_t* par_off,
                    size_t* offa_off, size_t* offf_off, size_t* offr_off) {
  size_t rs = hs[0]->cfg.prec == M1_FP32 ? sizeof(GridArgs<float>) : sizeof(GridArgs<double>);
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
  *args_off = take(2 * (size_t)n * rs);
  *par_off = take((size_t)n * sizeof(int));
  *offa_off = take((size_t)kNumBatchVariants * (n + 1) * sizeof(int));
  *offf_off = take((size_t)(n + 1) * sizeof(int));
  *offr_off = take((size_t)(n + 1) * sizeof(int));
  return off;
}

int check_members(m1_handle* const* hs, int n) {
  if (!hs || n <= 0) return fail(M1_EINVAL, "empty batch");
  for (int q = 0; q < n; ++q) {
    if (!hs[q]) return fail(M1_EINVAL, "handle %d is NULL", q);
    if (hs[q]->broken) return fail(M1_ESTATE, "handle %d had a device error", q);
    if (hs[q]->cfg.prec != hs[0]->cfg.prec) return fail(M1_EINVAL, "mixed precisions in a batch");
    if (hs[q]->stream != hs[0]->stream) return fail(M1_EINVAL, "batch members must share a stream");
    if (hs[q]->cfg.substep_rule)
      return fail(M1_EUNSUPPORTED, "handle %d uses the substep rule: step it alone", q);
    if (hs[q]->cfg.flux != M1_FLUX_GLF)
      return fail(M1_EUNSUPPORTED, "handle %d uses the eigenvalue HLL flux: step it alone", q);
    if (hs[q]->band)
      return fail(M1_EUNSUPPORTED, "handle %d is a band grid: step it alone", q);
    for (int r = 0; r < q; ++r)
      if (hs[r] == hs[q]) return fail(M1_EINVAL, "handle %d appears twice", q);
  }
  return M1_OK;
}

template <typename R>
int upload_args(m1_batch* b) {
  std::vector<GridArgs<R>> args(2 * (size_t)b->n);
  for (int q = 0; q < b->n; ++q) {
    const GridArgs<R>* src = (b->prec == M1_FP32) ? (const GridArgs<R>*)b->hs[q]->af
                                                  : (const GridArgs<R>*)b->hs[q]->ad;
    args[q] = src[0];
    args[b->n + q] = src[1];
  }
  HIPCHK(hipMemcpyAsync(b->ws + b->args_off, args.data(), args.size() * sizeof(GridArgs<R>),
                        hipMemcpyHostToDevice, b->stream));
  HIPCHK(hipStreamSynchronize(b->stream));
  return M1_OK;
}

int sync_parity(m1_batch* b) {
  bool fresh = true;
  for (int q = 0; q < b->n; ++q)
    if (b->gen[q] != b->hs[q]->gen) fresh = false;
  if (!fresh) {               // a member's c_tilde changed: new descriptor table
    int st = b->prec == M1_FP32 ? upload_args<float>(b) : upload_args<double>(b);
    if (st) return st;
    for (int q = 0; q < b->n; ++q) b->gen[q] = b->hs[q]->gen;
    if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; b->graph_sp = -1; }
  }
  bool same = true;
  for (int q = 0; q < b->n; ++q)
    if ((b->par[q] ^ b->sp) != b->hs[q]->cur) same = false;
  if (same) return M1_OK;
  for (int q = 0; q < b->n; ++q) b->par[q] = b->hs[q]->cur ^ b->sp;
  HIPCHK(hipMemcpyAsync(b->ws + b->par_off, b->par.data(), b->n * sizeof(int),
                        hipMemcpyHostToDevice, b->stream));
  HIPCHK(hipStreamSynchronize(b->stream));
  if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; b->graph_sp = -1; }
  return M1_OK;
}

template <typename R>
hipError_t batch_launch_step(m1_batch* b, int variant) {
  const GridArgs<R>* args = (const GridArgs<R>*)(b->ws + b->args_off);
  const int* par = (const int*)(b->ws + b->par_off);
  const int* offa = (const int*)(b->ws + b->offa_off) + (size_t)variant * (b->n + 1);
  const int* offf = (const int*)(b->ws + b->offf_off);
  const int* offr = (const int*)(b->ws + b->offr_off);
  hipError_t e = hipSuccess;
  for (int q = 0; q < b->n && e == hipSuccess; ++q)
    e = launch_selection(b->hs[q], (b->par[q] ^ b->sp) & 1, b->stream);
  if (e == hipSuccess)
    e = launch_advect_batched<R>(variant, args, par, b->n, b->sp, offa, b->blocks_adv[variant],
                                 b->active, b->stream);
  if (e != hipSuccess || variant == kFusedVariant) return e;   // fused: no separate freq kernel
  return launch_freq_batched<R>(args, par, b->n, b->sp, offf, b->blocks_freq, b->islands, offr,
                                b->blocks_rates,
                                b->stream);
}

hipError_t batch_one_step(m1_batch* b, int variant) {
  hipError_t e = b->prec == M1_FP32 ? batch_launch_step<float>(b, variant)
                                    : batch_launch_step<double>(b, variant);
  if (e != hipSuccess) return e;
  b->sp ^= 1;
  for (auto* h : b->hs) { h->cur ^= 1; h->steps += 1; h->t += h->dt; }
  return hipSuccess;
}
}  // namespace

extern "C" {

int32_t m1_batch_workspace_bytes(m1_handle* const* hs, int32_t n, size_t* bytes) {
  if (!bytes) return fail(M1_EINVAL, "bytes is NULL");
  int st = check_members(hs, n);
  if (st) return st;
  size_t a, p, oa, of;
  size_t orr;
  *bytes = batch_layout(hs, n, &a, &p, &oa, &of, &orr);
  return M1_OK;
}

int32_t m1_batch_init(m1_handle* const* hs, int32_t n, void* d_ws, size_t ws_bytes,
                      int32_t use_graph, m1_batch** out) {
  if (!out) return fail(M1_EINVAL, "out is NULL");
  *out = nullptr;
  int st = check_members(hs, n);
  if (st) return st;
  if (!d_ws || (((uintptr_t)d_ws) & 255)) return fail(M1_EINVAL, "workspace NULL or not 256-byte aligned");
  m1_batch* b = new m1_batch();
  b->hs.assign(hs, hs + n);
  b->n = n;
  b->prec = hs[0]->cfg.prec;
  b->stream = hs[0]->stream;
  b->ws = (char*)d_ws;
  size_t need = batch_layout(hs, n, &b->args_off, &b->par_off, &b->offa_off, &b->offf_off,
                             &b->offr_off);
  if (ws_bytes < need) { delete b; return fail(M1_ENOMEM, "batch workspace %zu < %zu", ws_bytes, need); }
  b->use_graph = use_graph != 0 && b->stream != nullptr;
  for (int q = 0; q < n; ++q)
    if (hs[q]->cfg.prec == M1_FP32 && hs[q]->cfg.fp64_tau < INFINITY) b->islands = 1;
  b->fused_ok = b->prec == M1_FP32 && !b->islands;
  // work lists: prefix sums of work items per grid, per tile variant
  std::vector<int> offa((size_t)kNumBatchVariants * (n + 1)), offf(n + 1, 0), offr(n + 1, 0);
  int64_t tot[kNumBatchVariants] = {};
  for (int v = 0; v < kNumBatchVariants; ++v) {
    offa[(size_t)v * (n + 1)] = 0;
    for (int q = 0; q < n; ++q) {
      tot[v] += advect_blocks(hs[q]->cfg.nx, hs[q]->cfg.ny, hs[q]->nb, kBatchBK[v]);
      if (tot[v] > INT32_MAX / 2) { delete b; return fail(M1_EUNSUPPORTED, "batch too large"); }
      offa[(size_t)v * (n + 1) + q + 1] = (int)tot[v];
    }
  }
  int64_t totf = 0, totr = 0;
  for (int q = 0; q < n; ++q) {
    totf += freq_blocks(hs[q]->cfg.nx, hs[q]->cfg.ny);
    offf[q + 1] = (int)totf;
    totr += ((int64_t)(hs[q]->nb - 1) * (int64_t)hs[q]->nc + 255) / 256;
    if (totr > INT32_MAX / 2) { delete b; return fail(M1_EUNSUPPORTED, "batch too large"); }
    offr[q + 1] = (int)totr;
  }
  for (int q = 0; q < n; ++q)
    if (hs[q]->cfg.active_frac > 0.0) b->active = 1;
  // a block per work item (capped; the kernels stride over any rest)
  constexpr int64_t kMaxBlocks = int64_t(1) << 30;
  for (int v = 0; v < kNumBatchVariants; ++v) b->blocks_adv[v] = (int)std::min(tot[v], kMaxBlocks);
  b->blocks_freq = (int)std::min(totf, kMaxBlocks);
  b->blocks_rates = (int)std::min(totr, kMaxBlocks);
  b->par.resize(n);
  for (int q = 0; q < n; ++q) b->par[q] = hs[q]->cur;
  b->sp = 0;
  hipError_t e = hipMemcpyAsync(b->ws + b->offa_off, offa.data(), offa.size() * sizeof(int),
                                hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->ws + b->offr_off, offr.data(), offr.size() * sizeof(int),
                       hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->ws + b->offf_off, offf.data(), offf.size() * sizeof(int),
                       hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->ws + b->par_off, b->par.data(), n * sizeof(int), hipMemcpyHostToDevice,
                       b->stream);
  if (e != hipSuccess) { delete b; return fail(M1_EDEVICE, "batch upload: %s", hipGetErrorString(e)); }
  b->gen.resize(n);
  for (int q = 0; q < n; ++q) b->gen[q] = hs[q]->gen;
  st = b->prec == M1_FP32 ? upload_args<float>(b) : upload_args<double>(b);
  if (st) { delete b; return st; }
  *out = b;
  return M1_OK;
}

int32_t m1_batch_step(m1_batch* b, int32_t nsteps) {
  if (!b) return fail(M1_EINVAL, "batch is NULL");
  if (nsteps < 0) return fail(M1_EINVAL, "nsteps < 0");
  for (auto* h : b->hs)
    if (h->broken) return fail(M1_ESTATE, "a batch member had a device error");
  int st = sync_parity(b);
  if (st) return st;
  int left = nsteps;
  // autotuning on real steps: time each variant's steps with events
  auto skip_unusable = [&]() {
    if (b->variant < 0 && b->trial_variant == kFusedVariant && !b->fused_ok) {
      b->trial_ms[kFusedVariant] = INFINITY;
      b->trial_variant = kNumBatchVariants;
    }
    if (b->variant < 0 && b->trial_variant == kNumBatchVariants) {
      int best = 0;
      for (int v = 1; v < kNumBatchVariants; ++v)
        if (b->trial_ms[v] < b->trial_ms[best]) best = v;
      b->variant = best;
    }
  };
  skip_unusable();
  while (left > 0 && b->variant < 0) {
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, b->stream));
    hipError_t e = batch_one_step(b, b->trial_variant);
    if (e != hipSuccess) { b->hs[0]->broken = true; return fail(M1_EDEVICE, "batch step: %s", hipGetErrorString(e)); }
    HIPCHK(hipEventRecord(e1, b->stream));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (b->trial_step > 0) b->trial_ms[b->trial_variant] += ms;   // first step warms up
    --left;
    if (++b->trial_step == kTrialSteps + 1) {
      b->trial_ms[b->trial_variant] /= kTrialSteps;
      b->trial_step = 0;
      ++b->trial_variant;
      skip_unusable();
    }
  }
  while (left > 0) {
    if (b->use_graph && left >= 2) {
      if (!b->exec || b->graph_sp != b->sp) {
        if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        int sp0 = b->sp;
        hipError_t e1 = b->prec == M1_FP32 ? batch_launch_step<float>(b, b->variant)
                                           : batch_launch_step<double>(b, b->variant);
        b->sp ^= 1;
        hipError_t e2 = e1 == hipSuccess ? (b->prec == M1_FP32 ? batch_launch_step<float>(b, b->variant)
                                                               : batch_launch_step<double>(b, b->variant))
                                         : e1;
        b->sp = sp0;
        hipError_t ec = hipStreamEndCapture(b->stream, &g);
        if (e2 != hipSuccess || ec != hipSuccess) {
          if (g) (void)hipGraphDestroy(g);
          return fail(M1_EDEVICE, "graph capture failed: %s", hipGetErrorString(e2 != hipSuccess ? e2 : ec));
        }
        hipError_t ei = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) { b->exec = nullptr; return fail(M1_EDEVICE, "graph instantiate: %s", hipGetErrorString(ei)); }
        b->graph_sp = b->sp;
      }
      HIPCHK(hipGraphLaunch(b->exec, b->stream));
      for (int r = 0; r < 2; ++r)
        for (auto* h : b->hs) { h->cur ^= 1; h->steps += 1; h->t += h->dt; }
      left -= 2;
    } else {
      hipError_t e = batch_one_step(b, b->variant);
      if (e != hipSuccess) { b->hs[0]->broken = true; return fail(M1_EDEVICE, "batch step: %s", hipGetErrorString(e)); }
      --left;
    }
  }
  return M1_OK;
}

int32_t m1_batch_info(const m1_batch* b, int32_t* bins_per_block, double* ms, int32_t nv) {
  if (!b) return fail(M1_EINVAL, "batch is NULL");
  if (bins_per_block) *bins_per_block = b->variant >= 0 ? kBatchBK[b->variant] : 0;
  for (int v = 0; ms && v < nv && v < kNumBatchVariants; ++v) ms[v] = b->trial_ms[v];
  return M1_OK;
}

int32_t m1_batch_set_tile(m1_batch* b, int32_t bins_per_block) {
  if (!b) return fail(M1_EINVAL, "batch is NULL");
  for (int v = 0; v < kNumBatchVariants; ++v)
    if (kBatchBK[v] == bins_per_block) {
      if (v == kFusedVariant && !b->fused_ok)
        return fail(M1_EUNSUPPORTED, "the fused kernel needs FP32 grids without island cells");
      b->variant = v;
      return M1_OK;
    }
  return fail(M1_EINVAL, "no tile variant with %d bins per block", bins_per_block);
}

int32_t m1_batch_workspace_bound(int32_t n, int32_t prec, size_t* bytes) {
  if (!bytes || n <= 0 || (prec != M1_FP32 && prec != M1_FP64)) return fail(M1_EINVAL, "bad arguments");
  size_t rs = prec == M1_FP32 ? sizeof(GridArgs<float>) : sizeof(GridArgs<double>);
  *bytes = align_up(2 * (size_t)n * rs) + align_up((size_t)n * sizeof(int)) +
           align_up((size_t)kNumBatchVariants * (n + 1) * sizeof(int)) +
           2 * align_up((size_t)(n + 1) * sizeof(int));
  return M1_OK;
}

int32_t m1_batch_free(m1_batch* b) {
  if (b) (void)hipStreamSynchronize(b->stream);   // launches in flight read the workspace
  if (b && b->exec) (void)hipGraphExecDestroy(b->exec);
  delete b;
  return M1_OK;
}

int32_t m1_sync(m1_handle* h) {
  if (!h) return fail(M1_EINVAL, "handle is NULL");
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    h->broken = true;
    return fail(M1_EDEVICE, "stream error: %s", hipGetErrorString(e));
  }
  return M1_OK;
}

int32_t m1_residual(m1_handle* h, double* resid) {
  if (!h || !resid) return fail(M1_EINVAL, "bad arguments");
  if (h->steps == 0) { *resid = INFINITY; return M1_OK; }
  size_t n = (size_t)h->nb * h->nc;
  int nblk = (int)std::min<size_t>((n + 255) / 256, kResBlocks);
  double* part = (double*)(h->ws + h->L.partial);
  double* res = (double*)(h->ws + h->L.result);
  const char* Eold = h->ws + h->L.state[h->cur ^ 1][0];
  const char* Enew = h->ws + h->L.state[h->cur][0];
  hipError_t e = h->cfg.prec == M1_FP32
      ? launch_residual<float>((const float*)Eold, (const float*)Enew, n, part, nblk, res, h->stream)
      : launch_residual<double>((const double*)Eold, (const double*)Enew, n, part, nblk, res, h->stream);
  if (e != hipSuccess) return fail(M1_EDEVICE, "residual launch: %s", hipGetErrorString(e));
  double r2[2];
  HIPCHK(hipMemcpyAsync(r2, res, sizeof r2, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  *resid = r2[1] > 0 ? sqrt(r2[0] / r2[1]) : (r2[0] == 0 ? 0.0 : INFINITY);
  return M1_OK;
}

int32_t m1_residuals(m1_handle* const* hs, int32_t n, double* resid) {
  if (!hs || n < 1 || !resid) return fail(M1_EINVAL, "bad arguments");
  for (int q = 0; q < n; ++q)
    if (!hs[q]) return fail(M1_EINVAL, "handle %d is NULL", q);
  // every reduction first, then the copies (the first waits for them all on
  // a shared stream), then one wait per handle
  std::vector<double> r2(2 * (size_t)n, 0.0);
  for (int q = 0; q < n; ++q) {
    m1_handle* h = hs[q];
    if (h->steps == 0) continue;
    const size_t cnt = (size_t)h->nb * h->nc;
    const int nblk = (int)std::min<size_t>((cnt + 255) / 256, kResBlocks);
    double* part = (double*)(h->ws + h->L.partial);
    double* res = (double*)(h->ws + h->L.result);
    const char* Eold = h->ws + h->L.state[h->cur ^ 1][0];
    const char* Enew = h->ws + h->L.state[h->cur][0];
    hipError_t e = h->cfg.prec == M1_FP32
        ? launch_residual<float>((const float*)Eold, (const float*)Enew, cnt, part, nblk, res, h->stream)
        : launch_residual<double>((const double*)Eold, (const double*)Enew, cnt, part, nblk, res, h->stream);
    if (e != hipSuccess) return fail(M1_EDEVICE, "residual launch: %s", hipGetErrorString(e));
  }
  for (int q = 0; q < n; ++q) {
    m1_handle* h = hs[q];
    if (h->steps == 0) continue;
    HIPCHK(hipMemcpyAsync(&r2[2 * (size_t)q], h->ws + h->L.result, 2 * sizeof(double),
                          hipMemcpyDeviceToHost, h->stream));
  }
  for (int q = 0; q < n; ++q) {
    hipError_t e = hipStreamSynchronize(hs[q]->stream);
    if (e != hipSuccess) {
      hs[q]->broken = true;
      return fail(M1_EDEVICE, "stream error: %s", hipGetErrorString(e));
    }
  }
  for (int q = 0; q < n; ++q) {
    const double num = r2[2 * (size_t)q], den = r2[2 * (size_t)q + 1];
    resid[q] = hs[q]->steps == 0 ? INFINITY
                                 : (den > 0 ? sqrt(num / den) : (num == 0 ? 0.0 : INFINITY));
  }
  return M1_OK;
}

int32_t m1_solve_steady(m1_handle* h, double rel_tol, int64_t max_steps, int32_t check_every,
                        int64_t* steps_done, double* resid) {
  if (!h) return fail(M1_EINVAL, "handle is NULL");
  if (!(rel_tol > 0) || max_steps < 1 || check_every < 1) return fail(M1_EINVAL, "bad arguments");
  int64_t done = 0;
  double r = INFINITY;
  int st = M1_OK;
  while (done < max_steps) {
    int32_t n = (int32_t)std::min<int64_t>(check_every, max_steps - done);
    st = m1_step(h, n, nullptr);
    if (st) break;
    done += n;
    st = m1_residual(h, &r);
    if (st) break;
    if (r < rel_tol) break;
  }
  if (steps_done) *steps_done = done;
  if (resid) *resid = r;
  if (st) return st;
  if (!(r < rel_tol)) return fail(M1_ENOTCONV, "residual %.3e after %lld steps", r, (long long)done);
  return M1_OK;
}

}  // extern "C"

namespace {
// Physical state of the window [i0, i1) x [j0, j1) of every bin.
int state_out(m1_handle* h, int i0, int i1, int j0, int j1, double* d_E, double* d_Fx,
              double* d_Fy) {
  const char* E = h->ws + h->L.state[h->cur][0];
  const char* fx = h->ws + h->L.state[h->cur][1];
  const char* fy = h->ws + h->L.state[h->cur][2];
  hipError_t e = h->cfg.prec == M1_FP32
      ? launch_state_out<float>((const float*)E, (const float*)fx, (const float*)fy, h->cfg.nx,
                                h->cfg.ny, h->nb, i0, j0, i1 - i0, j1 - j0, -h->e2, d_E, d_Fx,
                                d_Fy, h->stream)
      : launch_state_out<double>((const double*)E, (const double*)fx, (const double*)fy,
                                 h->cfg.nx, h->cfg.ny, h->nb, i0, j0, i1 - i0, j1 - j0, -h->e2,
                                 d_E, d_Fx, d_Fy, h->stream);
  if (e != hipSuccess) return fail(M1_EDEVICE, "copy launch: %s", hipGetErrorString(e));
  return m1_sync(h);
}
}  // namespace

extern "C" {

int32_t m1_get_state(m1_handle* h, double* d_E, double* d_Fx, double* d_Fy) {
  if (!h) return fail(M1_EINVAL, "handle is NULL");
  return state_out(h, 0, h->cfg.nx, 0, h->cfg.ny, d_E, d_Fx, d_Fy);
}

int32_t m1_get_state_region(m1_handle* h, int32_t i0, int32_t i1, int32_t j0, int32_t j1,
                            double* d_E, double* d_Fx, double* d_Fy) {
  if (!h) return fail(M1_EINVAL, "handle is NULL");
  if (i0 < 0 || j0 < 0 || i1 > h->cfg.nx || j1 > h->cfg.ny || i0 >= i1 || j0 >= j1)
    return fail(M1_EINVAL, "region [%d,%d) x [%d,%d) outside the %d x %d grid or empty", i0, i1,
                j0, j1, h->cfg.nx, h->cfg.ny);
  return state_out(h, i0, i1, j0, j1, d_E, d_Fx, d_Fy);
}

int32_t m1_set_state(m1_handle* h, const double* d_E, const double* d_Fx, const double* d_Fy) {
  if (!h || !d_E || !d_Fx || !d_Fy) return fail(M1_EINVAL, "bad arguments");
  size_t n = (size_t)h->nb * h->nc;
  char* E = h->ws + h->L.state[h->cur][0];
  char* fx = h->ws + h->L.state[h->cur][1];
  char* fy = h->ws + h->L.state[h->cur][2];
  hipError_t e = h->cfg.prec == M1_FP32
      ? launch_state_in<float>(d_E, d_Fx, d_Fy, n, h->e2, (float*)E, (float*)fx, (float*)fy,
                               h->stream)
      : launch_state_in<double>(d_E, d_Fx, d_Fy, n, h->e2, (double*)E, (double*)fx, (double*)fy,
                                h->stream);
  if (e != hipSuccess) return fail(M1_EDEVICE, "copy launch: %s", hipGetErrorString(e));
  return M1_OK;
}

int32_t m1_force(m1_handle* h, double* fx, double* fy, double* gx, double* gy) {
  if (!h) return fail(M1_EINVAL, "handle is NULL");
  hipError_t e = launch_force_out((const double*)(h->ws + h->L.force), h->nc, -h->e2, fx, fy, gx,
                                  gy, h->stream);
  if (e != hipSuccess) return fail(M1_EDEVICE, "force launch: %s", hipGetErrorString(e));
  return M1_OK;
}

int32_t m1_free(m1_handle* h) {
  delete h;
  return M1_OK;
}

}  // extern "C"
