// Launch wrappers of the device kernels (host side).
#pragma once
#include <hip/hip_runtime.h>
#include <algorithm>
#include <stddef.h>
#include <stdint.h>

#include "m1_device.h"

namespace m1 {

// ---- hot path (m1_step_kernels.hip)
template <typename R>
hipError_t launch_step(const GridArgs<R>& a, hipStream_t s);
// Tiles of a grid (32 x 16 cells each).
int tile_count(int nx, int ny);
template <typename R>
hipError_t launch_advect(const GridArgs<R>& a, hipStream_t s);
template <typename R>
hipError_t launch_freq(const GridArgs<R>& a, hipStream_t s);
// Step of a grid of broad bands: advection + emission/absorption + force,
// one block per tile walking every band.
template <typename R>
hipError_t launch_band_step(const GridArgs<R>& a, hipStream_t s);
// ---- batched persistent launches (one launch per kernel and step for a
//      set of grids); variant selects the bins-per-block run length, or the
//      fused kernel (kBatchBK = -1: a block walks all bins of a tile)
constexpr int kNumBatchVariants = 5;
constexpr int kFusedVariant = 4;
extern const int kBatchBK[kNumBatchVariants];
int advect_blocks(int nx, int ny, int nb, int bk);
int freq_blocks(int nx, int ny);
template <typename R>
hipError_t launch_advect_batched(int variant, const GridArgs<R>* args, const int* par, int n,
                                 int sp, const int* off, int nblocks, int active, hipStream_t s);
// off/nblocks: 256-cell work items; offr/nrates: 256-interface work items of
// the two-launch step a batch of few cells takes.
template <typename R>
hipError_t launch_freq_batched(const GridArgs<R>* args, const int* par, int n, int sp,
                               const int* off, int nblocks, int islands, const int* offr,
                               int nrates, hipStream_t s);

// Active bins of a state E [nb][ny][nx]: per-bin energies with cell volumes
// wx[i] wy[j] into part [nb][energy_chunks], then flags active[k].
int energy_chunks(size_t nc);
template <typename R>
hipError_t launch_active_bins(const R* E, int nx, int ny, int nb, const double* wx,
                              const double* wy, const double* dnu, double frac, double* part,
                              int32_t* active, hipStream_t s);

template <typename R>
hipError_t launch_residual(const R* E0, const R* E1, size_t n, double* partial, int nblk,
                           double* out, hipStream_t s);
// Physical FP64 state (E, F) of a window of every bin from the internal (E, f)
// state, and the internal state from a physical one.
template <typename S>
hipError_t launch_state_out(const S* E, const S* fx, const S* fy, int nx, int ny, int nb, int i0,
                            int j0, int w, int h, int e2, double* dE, double* dFx, double* dFy,
                            hipStream_t s);
template <typename D>
hipError_t launch_state_in(const double* sE, const double* sFx, const double* sFy, size_t n,
                           int e2, D* E, D* fx, D* fy, hipStream_t s);
hipError_t launch_force_out(const double* force, size_t nc, int e2, double* fx, double* fy,
                            double* gx, double* gy, hipStream_t s);

// ---- set-up (m1_setup_kernels.hip)
// Bin-averaged Voigt profile of every temperature class (FP64):
// hbar[cls][k], emission profile phi = hbar / sum_k dnu_k hbar_k.
template <typename R>
hipError_t launch_class_profiles(const double* dnuD, const double* av, int64_t ncls,
                                 const double* dnu_edges, const double* dnu, int nb,
                                 const double* dawson_nodes, double* tmp, R* hbar, R* phi,
                                 hipStream_t s);

struct CellInputs {
  const double *n_HI, *T, *ux, *uy, *acabs, *acF, *pd, *emis;
};

// Per-cell opacities and emission (scaled by 2^e2 / c), island flags.
template <typename R>
hipError_t launch_cell_setup(const CellInputs& in, size_t nc, double dmin, double fp64_tau,
                             int e2, R* alpha, R* acF, R* acabs, R* pda, R* em,
                             uint8_t* island, hipStream_t s);

// Face-normal and tangential mean velocities of x- and y-faces (FP64 temp),
// then cell velocity gradients and face-normal velocities in R.
template <typename R>
hipError_t launch_velocity(const CellInputs& in, int nx, int ny, int geom, const int* bc,
                           const double* xe, const double* ye, double* tmp, R* ufx, R* ufy,
                           R* grad, hipStream_t s);

// Block maxima of the dynamic reduced-speed-of-light term (cs: sound speed).
hipError_t launch_dyn_rsl(const CellInputs& in, const double* cs, size_t nc, double dmax,
                          double* partial, int nblk, hipStream_t s);
// Maximum of n doubles on the device (NaN if any is NaN) into *out.
hipError_t launch_max_of(const double* partial, int n, double* out, hipStream_t s);

// Block partials of max |u|, max emis, min T (for dt and the state scale).
hipError_t launch_init_reduce(const CellInputs& in, size_t nc, double* partial, int nblk,
                              hipStream_t s);

}  // namespace m1
