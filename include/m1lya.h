/*
 * m1lya.h -- C ABI of the MI355X M1 Lyman-alpha transfer step.
 *
 * The method is the two-moment (M1) Lyman-alpha radiative-transfer step of
 * Nebrin et al. (arXiv 2606.02711), Section 2.1 and Appendix A:
 *   - Levermore closure of the Eddington tensor (Section 2.1, M1 closure);
 *   - frequency grid of N_nu bins geometric in nu - nu_Lya (Section 2.1);
 *   - explicit advection step: MinMod-limited linear reconstruction of J and
 *     f = H/J, GLF interface flux (= HLL with signal speeds +-c_tilde) blended
 *     with the diffusion flux by eps(tau) (Section 2.1, corrected GLF flux),
 *     upwind velocity advection and radiation-pressure work term;
 *   - implicit emission / absorption / destruction step (Section 2.1, BDF1);
 *   - radiation force density handed to hydrodynamics (Section 2.3);
 *   - implicit frequency step: Fokker-Planck diffusion, recoil and Doppler
 *     shift with the exponential scheme and a per-cell tridiagonal solve
 *     (Appendix A), H rescaled by J_new / J_old;
 *   - RT time step from the CFL condition (Section 2.1).
 *
 * Conventions common to every entry point
 *   - Every function returns an m1_status; nothing aborts or throws across
 *     the ABI.  m1_last_error() returns a thread-local message for the last
 *     failure of the calling thread.
 *   - Pointers named d_* are device pointers (hipMalloc'd memory or a torch
 *     CUDA tensor's data_ptr()).  The library never allocates device memory:
 *     all device state lives in the caller's workspace (see
 *     m1_workspace_bytes), which is what makes admission by HBM budget exact.
 *     The handle itself is a small host allocation released by m1_free.
 *   - Cell arrays are [ny][nx] with index j*nx + i; x is R and y is z in
 *     cylindrical geometry.  Per-bin arrays are [N_nu][ny][nx].
 *   - State E_k = 4 pi J_k / c and F_k = 4 pi H_k / c (per Hz, cgs): the
 *     spectral radiation energy density and flux over c, bin averaged.
 *   - Work is enqueued on the handle's stream and is asynchronous unless
 *     stated otherwise.  Device faults surface at m1_sync, m1_get_state,
 *     m1_solve_steady (which synchronise).
 *   - A handle is not thread safe.  Distinct handles on distinct streams may
 *     run concurrently.
 */
#ifndef M1LYA_H
#define M1LYA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  M1_OK = 0,
  M1_EINVAL = -1,        /* invalid argument (validated before any device work) */
  M1_ENOMEM = -2,        /* workspace smaller than m1_workspace_bytes */
  M1_EDEVICE = -3,       /* a HIP runtime call or kernel failed */
  M1_ENOTCONV = -4,      /* m1_solve_steady reached max_steps */
  M1_ESTATE = -5,        /* handle in an unusable state */
  M1_EUNSUPPORTED = -6   /* valid request the library does not implement */
} m1_status;

typedef enum { M1_CART2D = 0, M1_CYL_RZ = 1 } m1_geom;
typedef enum { M1_BC_VACUUM = 0, M1_BC_REFLECT = 1 } m1_bc;
/* State storage and arithmetic.  M1_FP64: everything in double.  M1_FP32:
 * state, opacities and transport arithmetic in float; in the frequency step
 * the exponential-scheme coefficients are computed in float, or in double in
 * cells whose line-centre optical depth exceeds fp64_tau, and the
 * (subtraction-free) elimination always runs in double; force sums and
 * residual norms are double.  A step rounds the FP32 state once (the
 * changes of the transport and source steps are summed first), so the error
 * does not grow with the step count.  Measured against M1_FP64 on the
 * 512 x 1024 cylindrical workload after 1000 steps, relative L2 on E / F /
 * force: 6e-8 / 2e-7 / 4e-8 from E = F = 0, 3e-7 / 3e-6 / 7e-7 from a
 * developed radiation field. */
typedef enum { M1_FP64 = 0, M1_FP32 = 1 } m1_prec;

/* Interface flux of the advection step (Section 2.1).  M1_FLUX_GLF: the
 * corrected GLF flux the paper adopts (HLL with signal speeds -c_tilde and
 * +c_tilde, blended with the diffusion flux by eps(tau)).  M1_FLUX_HLL_EIG:
 * the HLL flux the paper reports having tried (footnote to its choice of the
 * GLF solver), with the extreme eigenvalues of the M1 system's flux Jacobian
 * along the face normal as signal speeds (Davis estimates over the two face
 * states; the paper gives no speeds, they are computed here from the
 * Levermore closure) and the same eps blend: the HLL dissipation of the F
 * flux scaled by eps, the whole E flux by eps plus (1 - eps) times the
 * diffusion flux.  A comparison variant: single-grid stepping only, without
 * active bins or substeps; batches, band grids and batched servers refuse it
 * (M1_EUNSUPPORTED). */
typedef enum { M1_FLUX_GLF = 0, M1_FLUX_HLL_EIG = 1 } m1_flux;

typedef struct {
  int32_t geom;            /* m1_geom.  Cylindrical requires x0 == 0 with a
                              reflecting x- (axis) boundary. */
  int32_t nx, ny;          /* cells, each >= 4 */
  double x0, x1, y0, y1;   /* domain edges [cm], uniform spacing */
  int32_t bc[4];           /* m1_bc for x-, x+, y-, y+ */
  double T_min;            /* frequency resolution temperature [K] (30) */
  double q;                /* bin growth factor (1.1) */
  double half_width;       /* grid half-width in dnu_D(T_min) units (1e5) */
  double c_tilde;          /* reduced speed of light [cm/s], 0 < c_tilde <= c */
  double cfl;              /* CFL factor, 0 < cfl <= 1 (0.4) */
  int32_t recoil;          /* 0/1: atomic recoil term of the frequency step */
  int32_t doppler;         /* 0/1: Doppler term of the frequency step */
  int32_t prec;            /* m1_prec */
  double fp64_tau;         /* FP32 only: line-centre cell optical depth above
                              which a cell's frequency-step coefficients are
                              computed in double (+inf: none, the default;
                              0: all cells) */
  double active_frac;      /* active-bin advection (Section 2.2; the paper
                              uses 1e-10): at the start of
                              every step bin k's energy in the volume,
                              W_k = dnu_k sum_cells dV E_k, is summed in double,
                              and only bins with W_k > active_frac sum_k W_k
                              are advected; the others keep their state
                              through the transport step, while emission/
                              absorption and the frequency step act on every
                              bin.  0 (the default): every bin is advected.
                              Must be >= 0.  Results then depend on the
                              selection, which is taken on the state in its
                              storage precision (FP32 and FP64 paths can differ
                              for a bin whose share sits at the threshold). */
  int32_t substep_rule;    /* 0/1: emission/absorption in substeps (Section
                              2.1, step 2): per cell, a substep is accepted
                              when the energy density sum_k dnu_k E_k changes
                              by less than 10 % of (e + e_floor), e_floor =
                              4 pi J_floor / c with J_floor = 1e-15 erg cm^-2
                              s^-1 sr^-1, and halved and redone otherwise; the
                              next substep tries twice the accepted length
                              (clipped to the time left); a substep of 2^-60
                              of the step or the 4096th attempt is accepted as
                              it is.  The force is the substep forces averaged
                              over the step.  0 (the default): one substep.
                              Single-grid stepping only (batches refuse such
                              handles with M1_EUNSUPPORTED). */
  int32_t flux;            /* an m1_flux value; M1_FLUX_GLF is the default */
} m1_config;

/* Per-cell physical inputs, FP64, [ny][nx].  Host pointers when on_device is
 * 0, device pointers otherwise.  Read once by m1_init; the library keeps no
 * reference to them afterwards. */
typedef struct {
  const double *n_HI;        /* neutral hydrogen density [cm^-3], >= 0 */
  const double *T;           /* gas temperature [K], > 0 */
  const double *u_x, *u_y;   /* gas velocity [cm/s] */
  const double *alpha_abs;   /* continuum absorption alpha_c (1 - omega) [cm^-1] */
  const double *alpha_flux;  /* continuum flux opacity alpha_c (1 - omega g) [cm^-1] */
  const double *p_d;         /* Lya destruction probability per scattering, >= 0 */
  const double *emis;        /* Lya luminosity density [erg s^-1 cm^-3], >= 0,
                                emitted with the normalised Voigt profile */
  int32_t on_device;
} m1_fields;

typedef struct m1_handle m1_handle;

/* Fills *cfg with the paper's defaults (T_min 30 K, q 1.1, half-width 1e5,
 * CFL 0.4, recoil and Doppler on, FP64, fp64_tau +inf, vacuum boundaries,
 * the GLF flux). */
int32_t m1_default_config(m1_config *cfg);

/* Number of frequency bins of cfg's grid (194 with the defaults; Section 2.1). */
int32_t m1_num_bins(const m1_config *cfg, int32_t *n_nu);

/* The bins of cfg's grid (Section 2.1: widths Delta nu_D(T_min) q^m outwards
 * from line centre, symmetric, the outermost clipped at the half-width):
 * nu_centre[k] the absolute centre frequency [Hz] (arithmetic midpoint of
 * the edges) and dnu[k] the width [Hz], k < m1_num_bins; host arrays, either
 * may be NULL.  Host-only (no device work); M1_EINVAL for an invalid cfg. */
int32_t m1_frequency_grid(const m1_config *cfg, double *nu_centre, double *dnu);

/* Exact device workspace bytes for cfg when the temperature field holds
 * n_temp_classes distinct values (pass 0 for the worst case, one per cell).
 * m1_count_temperature_classes gives that number for a host T array. */
int32_t m1_workspace_bytes(const m1_config *cfg, int64_t n_temp_classes, size_t *bytes);
int32_t m1_count_temperature_classes(const double *T_host, int64_t n, int64_t *n_classes);

/* The reduced speed of light chosen from the medium (Section 2.1, dynamic
 * RSL): c_dyn = 4 max over cells of max[1, (a_v tau_0)^(1/3) f_abs] max(|u|, c_s),
 * f_abs = 1 / (1 + (a_v tau_0)^(1/3) tau_c + 0.6 p_d tau_0), with tau_0 the
 * line-centre depth n_HI sigma_0(T) dmax and tau_c = alpha_abs dmax (dmax the
 * larger cell side of cfg); then c_tilde = min(max(100 km/s, c_dyn), c), and,
 * when c_prev > 0 (the previous value), at most a 25 % decrease or a factor 4
 * increase from it.  fields: device arrays (on_device = 1; emis and
 * alpha_flux unused); d_cs: device array of sound speeds [cm/s], ncell
 * doubles; d_work: at least 8192 bytes of caller device memory, 8-byte
 * aligned.  Runs on `stream` (NULL = default) and waits for it; *c_tilde
 * [cm/s] receives the result.  M1_EINVAL for NULL or host arrays, a NaN
 * c_prev or a non-finite term (T <= 0). */
int32_t m1_dynamic_c_tilde(const m1_config *cfg, const m1_fields *fields, const double *d_cs,
                           double c_prev, void *d_work, void *stream, double *c_tilde);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, the tight loop of a hydrodynamics driver, harnesses that forbid
 * allocation): m1_dynamic_c_tilde without d_work.  Its block maxima and their
 * maximum go to a static device array of the library, 8448 bytes on every GPU
 * the library runs on, held until the process ends; the call allocates
 * nothing (no device or host allocator).  It works on the current device
 * (stream, NULL = default, must belong to it) and returns the same value as
 * m1_dynamic_c_tilde, bitwise.  Every grid size fits the array (the kernel
 * strides over the cells).  Calls that overlap on one GPU (from other
 * threads, or on other streams) race on the array.  Argument checks and
 * errors as for m1_dynamic_c_tilde, plus M1_EDEVICE if the array's device
 * address cannot be obtained.  Waits for the stream. */
int32_t m1_dynamic_c_tilde_noalloc(const m1_config *cfg, const m1_fields *fields,
                                   const double *d_cs, double c_prev, void *stream,
                                   double *c_tilde);

/* Validates cfg and fields, lays out the caller-owned workspace d_ws of
 * ws_bytes (>= m1_workspace_bytes for the field's class count, 256-byte
 * aligned), runs the set-up kernels on `stream` (a hipStream_t; NULL =
 * default stream) and sets E = F = 0.  Synchronous.  On success *out
 * receives a new handle.  The set-up follows the paper: the frequency grid
 * of Section 2.1 (bins geometric in nu - nu_Lya from dnu_D(T_min)); the
 * bin-averaged Voigt profile <H>_k of Appendix A (second-order expansion in
 * a_v, evaluated exactly, no look-up table) per temperature class; the line
 * opacity alpha = n_HI sigma_0(T), the flux opacity alpha_F,k = alpha <H>_k +
 * alpha_c (1 - omega g) and the absorption alpha_c (1 - omega) + p_d alpha
 * <H>_k of Section 2.1 (steps 1 and 2); the emission profile <H>_k / sqrt(pi)
 * normalised over the grid; the velocity gradients of Appendix A (D : grad u
 * terms); the CFL time step of Section 2.1. */
int32_t m1_init(const m1_config *cfg, const m1_fields *fields, void *d_ws,
                size_t ws_bytes, void *stream, m1_handle **out);

/* Enqueues nsteps RT steps, each the three operator-split stages of Section
 * 2.1: (1) the explicit advection step (MinMod reconstruction of E and f,
 * Levermore closure, corrected GLF flux with the eps(tau) blend, upwind
 * velocity advection, radiation-pressure work term, hoop pressure in (R, z),
 * causality clamp), (2) the implicit emission/absorption/destruction step
 * (BDF1), with the force density of Section 2.3 formed from its result, and
 * (3) the implicit frequency step of Appendix A (exponential-scheme leakage
 * coefficients, tridiagonal BDF1 solve per cell, H rescaled by
 * J_new / J_old).  *t_now (may be NULL) receives the simulated time after
 * them.  Asynchronous on the handle's stream; M1_ESTATE after a device error. */
int32_t m1_step(m1_handle *h, int32_t nsteps, double *t_now);

/* Measurement variant of m1_step: records HIP events around every kernel
 * launch on the handle's stream, waits, and returns the summed device time
 * [ms] of the advection/emission-absorption kernel in ms[0] and of the
 * force/frequency-step kernel in ms[1] (nsteps <= 4096).  Same results as
 * m1_step; the events add only launch overhead. */
int32_t m1_step_profiled(m1_handle *h, int32_t nsteps, double *ms);

/* Enqueues a copy of the radiation force density of the last step (Section
 * 2.3: the momentum the radiation gives the gas and dust per unit volume,
 * sum_k dnu_k alpha_F,k F**_k in the state variables, equal to the paper's
 * form in the change of H over the absorption step) into caller device
 * arrays of ncell doubles [dyn cm^-3]: total (x, y) and the gas share (the
 * line opacity's part, the paper's eps_gas split; may be NULL).
 * Asynchronous. */
int32_t m1_force(m1_handle *h, double *d_fx, double *d_fy, double *d_fx_gas,
                 double *d_fy_gas);

/* Steps until r = ||E^{n+1} - E^n||_2 / ||E^{n+1}||_2 (all cells and bins,
 * FP64 sums) is below rel_tol, checking every check_every steps, or until
 * max_steps steps were taken by this call (then M1_ENOTCONV).  Blocking.
 * The paper runs its test clouds to a fixed time and reads results once they
 * have settled (Sections 3.1 and 3.3); this steady-state criterion is the
 * library's own stopping rule for the same solutions. */
int32_t m1_solve_steady(m1_handle *h, double rel_tol, int64_t max_steps,
                        int32_t check_every, int64_t *steps_done, double *resid);

/* Residual r of the last step (as in m1_solve_steady).  Blocking. */
int32_t m1_residual(m1_handle *h, double *resid);

/* m1_residual of n handles into resid[0..n-1] (host array), with every
 * reduction enqueued before the first wait: one synchronisation for handles
 * that share a stream (a serving round's residents).  Same values as n calls
 * of m1_residual.  Blocking.  M1_EINVAL for NULL arguments or n < 1. */
int32_t m1_residuals(m1_handle *const *hs, int32_t n, double *resid);

/* Copy the state out of / into caller device arrays of doubles
 * [N_nu][ny][nx] in physical units (E, F per Hz).  Internally the state is
 * E (scaled by 2^scale_exp2 in the FP32 path, see m1_get_info, so values far
 * below FLT_MIN are kept) and the reduced flux f = F/E in the state
 * precision: get forms F = f E in double (NULL outputs are skipped); set
 * stores f = F/E and drops the flux where E <= 0.  get is blocking; set is
 * asynchronous.  FP32 handles store E times 2^scale_exp2, a scale fixed at
 * init so that the first step's emission is of order one: a state set far
 * below that scale (below ~1e-30 of it) falls into float subnormals and
 * loses precision. */
int32_t m1_get_state(m1_handle *h, double *d_E, double *d_Fx, double *d_Fy);
int32_t m1_set_state(m1_handle *h, const double *d_E, const double *d_Fx,
                     const double *d_Fy);

/* Copy of the window i in [i0, i1), j in [j0, j1) of the state of every bin
 * into caller device arrays of doubles [N_nu][j1 - j0][i1 - i0] (physical
 * units; NULL outputs are skipped).  For grids whose full FP64 copy would not
 * fit beside the workspace.  Blocking. */
int32_t m1_get_state_region(m1_handle *h, int32_t i0, int32_t i1, int32_t j0, int32_t j1,
                            double *d_E, double *d_Fx, double *d_Fy);

/* Sets a grid's reduced speed of light to c_tilde (0 < c_tilde <= c), e.g.
 * the value m1_dynamic_c_tilde chose for the current medium (Section 2.1,
 * dynamic RSL), keeping the state: the time step becomes the CFL step of the
 * new c_tilde (m1_get_info reports it) and the geometry factors scaled by
 * c_tilde dt are rebuilt.  Line and band grids.  Waits for the handle's
 * stream (work already enqueued finishes with the old value).  A batch that
 * holds the handle uploads its new arguments at its next step.  M1_EINVAL
 * for a NULL handle or a c_tilde outside (0, c]; M1_ESTATE after a device
 * error. */
int32_t m1_set_c_tilde(m1_handle *h, double c_tilde);

/* Which bins the last step advected (Section 2.2, active bins):
 * flags_host[k] = 1 for an advected bin, 0 otherwise (N_nu int32 entries;
 * may be NULL), *n_active (may be NULL) their count.  With active_frac = 0
 * every bin is reported active; before the first step, none is.  Blocking
 * (waits for the handle's stream). */
int32_t m1_active_bins(m1_handle *h, int32_t *flags_host, int32_t *n_active);

/* Scalars of a handle: dt [s], N_nu, precision, cells, internal scale 2^e. */
int32_t m1_get_info(const m1_handle *h, double *dt, int32_t *n_nu, int32_t *prec,
                    int64_t *ncell, int32_t *scale_exp2);

/* ---- broad bands (Section 2.5 and Appendix E): the stellar bands (optical,
 * FUV, Lyman-Werner, EUV1-3) and the IR band move with the same M1 step:
 * the advection of Section 2.1 step 1 (MinMod reconstruction, Levermore
 * closure, corrected GLF flux whose blend eps(tau) takes tau from the band's
 * flux opacity, upwind velocity advection, work term, hoop pressure,
 * causality clamp) and the implicit emission/absorption of step 2, with no
 * frequency-derivative terms, so there is no frequency step.  Opacities and
 * emission come per band and cell from the caller, whose thermochemistry
 * (photoionisation, dust temperatures) sets them; it is not part of this
 * library.  A band grid is an m1_handle: m1_step, m1_step_profiled (all
 * time in ms[0]), m1_get_state, m1_get_state_region, m1_set_state (per band
 * instead of per Hz: E = 4 pi J_B / c, F = 4 pi H_B / c), m1_force, m1_residual,
 * m1_solve_steady, m1_active_bins (every band active), m1_get_info (N_nu =
 * number of bands), m1_sync and m1_free apply; batches refuse band grids. */

/* Per-band physical inputs, FP64.  Host pointers when on_device is 0,
 * device pointers otherwise; read once by m1_band_init. */
typedef struct {
  const double *u_x, *u_y;    /* gas velocity [cm/s], [ny][nx], |u| < c */
  const double *kappa_abs;    /* absorption opacity [cm^-1], [n_band][ny][nx], >= 0 */
  const double *kappa_flux;   /* flux-mean opacity [cm^-1] (sets eps(tau) and the
                                 force), [n_band][ny][nx], >= 0 */
  const double *emis;         /* luminosity density [erg s^-1 cm^-3], [n_band][ny][nx],
                                 >= 0; the E equation gains emis / c per unit length */
  int32_t on_device;
} m1_band_fields;

/* Exact device workspace bytes of a grid of n_band bands (1..1024) for cfg. */
int32_t m1_band_workspace_bytes(const m1_config *cfg, int32_t n_band, size_t *bytes);

/* As m1_init, for n_band broad bands.  cfg supplies the grid, boundaries,
 * c_tilde, cfl and precision (its frequency-grid, recoil, Doppler and
 * fp64_tau fields are validated as for m1_init and otherwise unused);
 * active_frac and substep_rule must be 0 (M1_EUNSUPPORTED otherwise).  The
 * time step is the line grids' CFL step.  The force of a step (m1_force)
 * is sum_B kappa_F,B F_B; the line-share outputs are 0.  M1_EINVAL for NULL,
 * negative or non-finite inputs or |u| >= c, M1_ENOMEM for a short
 * workspace.  Synchronous; on success *out receives a new handle. */
int32_t m1_band_init(const m1_config *cfg, int32_t n_band, const m1_band_fields *fields,
                     void *d_ws, size_t ws_bytes, void *stream, m1_handle **out);

/* ---- batches: many grids advanced by one launch per kernel and step (a
 * throughput addition with no counterpart in the paper).
 * A batch groups n handles of the same precision on the same stream.  Its
 * descriptor tables live in a caller workspace of m1_batch_workspace_bytes
 * bytes (256-byte aligned); the library allocates no device memory.  Every
 * grid's result is bitwise identical to stepping it alone.
 *
 * Tile variants: 7, 14, 28 or 49 bins per advection block with the
 * frequency step in a second kernel, or -1: one fused kernel whose blocks
 * walk all bins of a 32 x 16 tile and run the frequency step of their cells
 * (FP32 batches without island cells only).
 *
 * m1_batch_step: the first steps of a new batch time each tile variant
 * on real steps, which give identical results for every variant, and keep
 * the fastest; afterwards pairs of steps are
 * replayed from a captured HIP graph when use_graph is set and the stream
 * is not the null stream.  Stepping a member handle on its own between
 * batch steps is allowed (the batch re-reads the ping-pong parities). */
typedef struct m1_batch m1_batch;
int32_t m1_batch_workspace_bytes(m1_handle *const *hs, int32_t n, size_t *bytes);
int32_t m1_batch_init(m1_handle *const *hs, int32_t n, void *d_ws, size_t ws_bytes,
                      int32_t use_graph, m1_batch **out);
int32_t m1_batch_step(m1_batch *b, int32_t nsteps);
/* Chosen tile variant (7, 14, 28, 49 or -1; 0 while tuning) and the
 * measured step time of each of the five variants [ms per step; +inf for a
 * variant that does not apply]. */
int32_t m1_batch_info(const m1_batch *b, int32_t *bins_per_block, double *ms_per_variant,
                      int32_t n_variants);
/* Waits for the stream, then releases the host object (not the workspace). */
int32_t m1_batch_free(m1_batch *b);
/* Fixes the tile variant (7, 14, 28, 49 or -1) and ends tuning; results do
 * not depend on it.  -1 on a batch it does not apply to: M1_EUNSUPPORTED. */
int32_t m1_batch_set_tile(m1_batch *b, int32_t bins_per_block);
/* Upper bound of m1_batch_workspace_bytes for any n handles of precision prec. */
int32_t m1_batch_workspace_bound(int32_t n, int32_t prec, size_t *bytes);

/* ---- serving: a continuous-batching engine for steady-state solves (a
 * serving addition with no counterpart in the paper).
 *
 * The engine owns nothing on the device but what the caller hands it: one
 * arena of arena_bytes (256-byte aligned) that is its HBM budget.  A request
 * is admitted when a free block of exactly m1_workspace_bytes(cfg, classes)
 * bytes exists in the arena (first fit) and fewer than max_resident
 * requests are resident; queued requests are taken in arrival order, and a
 * smaller one may pass a head that does not fit at most max_bypass times
 * before admission waits for the head.  At admission the engine calls
 * fields_cb(user, id, &fields) for the request's inputs and runs m1_init;
 * the arrays must stay valid until the m1_server_run call that admits the
 * request returns.  A callback status other than M1_OK fails the request.
 *
 * m1_server_run performs rounds.  In a round every resident request takes
 * min(check_every, max_steps - steps) steps (in batched mode all requests
 * whose share is check_every advance together in one batch;
 * otherwise one request at a time, in order) and then its residual is
 * computed; a request whose residual is below rel_tol, or that reached
 * max_steps, is finished.  This is the schedule of m1_solve_steady, so each
 * result is bitwise identical to solving the request alone.  A finished
 * request keeps its arena block (for m1_server_handle, then m1_get_state /
 * m1_force) until m1_server_release.  The engine is single threaded. */
typedef struct m1_server m1_server;

typedef struct {
  int32_t prec;            /* m1_prec of every request (m1_config.prec is overridden) */
  int32_t batched;         /* 1: residents advance in one batch per round; 0: one at a time */
  int32_t max_resident;    /* >= 1 */
  int32_t check_every;     /* steps per round and between residual checks, >= 1 */
  int32_t use_graph;       /* batched mode: replay step pairs from a HIP graph */
  int32_t max_bypass;      /* >= 0 */
} m1_server_config;

typedef int32_t (*m1_fields_cb)(void *user, int64_t id, m1_fields *out);

/* Request states reported by m1_server_poll. */
typedef enum {
  M1_REQ_QUEUED = 0, M1_REQ_RESIDENT = 1, M1_REQ_CONVERGED = 2, M1_REQ_NOT_CONVERGED = 3,
  M1_REQ_REJECTED = 4, M1_REQ_FAILED = 5
} m1_req_state;

typedef struct {
  int64_t id;
  int32_t state;           /* m1_req_state */
  int32_t error;           /* m1_status of a failed init or step, else M1_OK */
  int64_t steps;
  double residual;
  int64_t admit_round, finish_round;
  size_t ws_bytes;
} m1_request_info;

int32_t m1_server_create(const m1_server_config *cfg, void *d_arena, size_t arena_bytes,
                         void *stream, m1_fields_cb cb, void *user, m1_server **out);
/* Queues a request.  cfg is copied; n_temp_classes as for m1_workspace_bytes.
 * A request that cannot fit an empty arena is recorded as rejected (it is
 * reported by the next m1_server_poll) and *id still receives its id.  A
 * batched server refuses a config with substep_rule set (M1_EUNSUPPORTED,
 * nothing queued). */
int32_t m1_server_submit(m1_server *s, const m1_config *cfg, int64_t n_temp_classes,
                         double rel_tol, int64_t max_steps, int64_t *id);
/* Runs up to `rounds` rounds (admission, steps, residual checks; blocking)
 * and returns early when nothing is resident or queued.  *n_busy (may be
 * NULL) receives the number of queued plus resident requests afterwards. */
int32_t m1_server_run(m1_server *s, int32_t rounds, int32_t *n_busy);
/* Moves up to cap records of requests that finished (or were rejected or
 * failed) since the last poll into out; *n receives the count. */
int32_t m1_server_poll(m1_server *s, m1_request_info *out, int32_t cap, int32_t *n);
/* Handle of a resident or finished request (owned by the engine). */
int32_t m1_server_handle(m1_server *s, int64_t id, m1_handle **h);
/* Frees a finished request's arena block and handle. */
int32_t m1_server_release(m1_server *s, int64_t id);
/* Counters: queued, resident, finished and not released, rounds run; arena
 * bytes in use and the largest free block. */
int32_t m1_server_stats(const m1_server *s, int64_t *queued, int64_t *resident,
                        int64_t *finished, int64_t *rounds, size_t *arena_used,
                        size_t *largest_free);
/* Waits for the stream and releases every request and the engine. */
int32_t m1_server_free(m1_server *s);

int32_t m1_sync(m1_handle *h);         /* waits for the stream; surfaces faults */
int32_t m1_free(m1_handle *h);         /* frees the host handle, not the workspace */
const char *m1_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* M1LYA_H */
