// sq_dev.h -- device-side data layout shared by the host plan (sq_capi.cpp)
// and the gfx950 kernels (sq_recur.hip, sq_misc.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define SQ_FDM 6          // FD half order on the device (12th-order stencil)
#define SQ_MAX_SPECIES 4
#define SQ_NEAR_MAX 32    // images whose projector is nonzero at the node
#define SQ_KL_MAX 64      // Lanczos steps
#define SQ_REC 24         // per-node record: rho, e, K[9], N[9], e_nl, dV V rho, xc energy, xc stress
#define SQ_TILE 2         // nodes per tile edge for the image lists
#define SQ_GRAM_MAX 1024  // projector pairs (I <= J) with overlapping supports in one cube
#define SQ_CENSUS 8       // census ints per cell

// error bits raised by kernels
#define SQ_ERR_SLOTS 1u
#define SQ_ERR_IMAGES 2u
#define SQ_ERR_BOUNDS 4u
#define SQ_ERR_NEAR 8u
#define SQ_ERR_RANGE 16u   // a projection left the range of the fixed-point sums

struct SpecDev {
  double v_amp, v_sig, v_rc, p_sig, p_rc, gamma;
};

// One cell as the kernels see it.  All per-node arrays are indexed by the
// global node id g = node_base + q.
struct CellDev {
  int n[3];
  int m, nc, npl, K;
  int nimg;           // atom images of the cell (all that reach any cube)
  int ntile[3];       // tiles per axis (SQ_TILE nodes per edge)
  int nsp;
  int mq;             // Gauss-Chebyshev points of the coefficient integrals (0: per-node rule)
  int mu_mode;
  int krun;           // Lanczos steps run: K, or ceil(npl / 2) when more and the moments come from them
  long long Nd, node_base;
  double h, dV, kT, ne, vol, mu0;
  double L[3];
  double c2[SQ_FDM + 1], c1[SQ_FDM + 1];
  double ck[SQ_FDM + 1];    // kinetic stencil weights -c2[k] / (2 h^2)
  float ckf[SQ_FDM + 1];    // the same rounded to FP32
  float padf;
  SpecDev sp[SQ_MAX_SPECIES];
  const double* vloc;     // [Nd]
  const double* img;      // [nimg][4]: x, y, z (unwrapped), species
  const int* tile_ptr;    // [ntiles + 1]
  const int* tile_img;    // image ids per tile
};

// Device buffers of a plan (concatenated over cells).
struct PlanDev {
  const CellDev* cells;   // [ncell]
  double* lan;            // [Ntot][2 * SQ_KL_MAX]  alpha then beta
  int* lan_steps;         // [Ntot]
  double* bnd;            // [Ntot][4]  lam_lo, lam_hi, chi, zeta
  double* mom;            // [Ntot][mstride]
  double* coef;           // [Ntot][mstride]
  double* rec;            // [Ntot][SQ_REC]
  double* nq;             // [Ntot]  per-node electron count at the trial mu
  double* nqd;            // [Ntot]  its derivative in mu
  double* mus;            // [ncell][8] Fermi-level bisection state
  double* sums;           // [ncell][SQ_REC + 4] reduced records
  unsigned* err;          // [1]
  // Gram matrix of the projectors of each node's cube, upper triangle, pairs
  // with overlapping supports only (written by the Lanczos pass, read by the
  // moments and stress passes): value, (I | J << 16), count (-1: too many)
  double* gval;           // [Ntot][SQ_GRAM_MAX]
  unsigned* gidx;         // [Ntot][SQ_GRAM_MAX]
  int* gn;                // [Ntot]
  int mstride;
  int inject;             // sq_options.inject (error-path tests)
};

// mus layout: SQ_MU_STRIDE doubles per cell
#define SQ_MU_STRIDE 16
#define MU_LO 0      // bracket with N(lo) < N_e < N(hi)
#define MU_HI 1
#define MU_MID 2     // trial Fermi level of the next evaluation
#define MU_VAL 3     // result
#define MU_DONE 4    // 0 running, 1 done, 2 not bracketed, 3 update cap reached
#define MU_IT 5
#define MU_PHASE 6
#define MU_N 7       // last electron count
#define MU_FLO 8     // N(lo) - N_e (Illinois-scaled)
#define MU_FHI 9     // N(hi) - N_e (Illinois-scaled)
#define MU_SIDE 10   // end point replaced last: -1 lo, +1 hi
#define MU_WID 11    // bracket width at the last progress check

// One launch of a recurrence kernel over a group of nodes of equal cube
// width: the slot capacity needed per column (kc: the variant with the
// smallest capacity >= kc runs), the single-sweep form (fused: the node's
// Gram matrix is stored) and the launch form (counter != NULL: a persistent
// grid of `grid` workgroups, or as many as the device holds at once when
// grid <= 0, takes nodes from an atomic work counter, which the launcher
// clears first; else one workgroup per node).
struct RecLaunch {
  int nc, kc;
  bool fused;
  unsigned* counter;
  int grid;
};

extern "C++" {
// launchers (sq_recur.hip per cube width, sq_misc.hip)
hipError_t sq_launch_vloc(const CellDev* d_cell, const CellDev& h_cell, double* vloc, hipStream_t s);
hipError_t sq_launch_lanczos(const RecLaunch& R, const PlanDev& P, const long long* items,
                             const int* item_cell, long long nitems, hipStream_t s);
hipError_t sq_launch_gram(int nc, const PlanDev& P, const long long* items,
                          const int* item_cell, long long nitems, hipStream_t s);
hipError_t sq_launch_bounds(const PlanDev& P, const long long* items, const int* item_cell,
                            long long nitems, hipStream_t s);
hipError_t sq_launch_moments(const RecLaunch& R, bool fp64, const PlanDev& P,
                             const long long* items, const int* item_cell, long long nitems,
                             hipStream_t s);
hipError_t sq_launch_mu_init(const PlanDev& P, const int* cells, int ncells, const int* fixed_mode,
                             hipStream_t s);
hipError_t sq_launch_mu_eval(const PlanDev& P, const long long* items, const int* item_cell,
                             long long nitems, hipStream_t s);
hipError_t sq_launch_mu_step(const PlanDev& P, const int* cells, int ncells, hipStream_t s);
hipError_t sq_launch_coeffs(const PlanDev& P, const long long* items, const int* item_cell,
                            long long nitems, hipStream_t s);
hipError_t sq_launch_qmoments(const PlanDev& P, const long long* items, const int* item_cell,
                              long long nitems, hipStream_t s);
hipError_t sq_launch_stress(const RecLaunch& R, bool fp64, const PlanDev& P,
                            const long long* items, const int* item_cell, long long nitems,
                            hipStream_t s);
hipError_t sq_launch_census(int nc, const PlanDev& P, const long long* items, const int* item_cell,
                            long long nitems, int* stats, long long* pairs, hipStream_t s);
hipError_t sq_launch_fill_u32(unsigned* p, unsigned v, long long n, hipStream_t s);

// Static device scratch of the library (sq_misc.hip): SQ_STATIC_CELLS rows of
// SQ_REC + 4 doubles, one array per GPU for the life of the process, used by
// the entry point that allocates nothing.  sq_static_scratch() returns the
// current device's address of the array (looked up once per device).
#define SQ_STATIC_CELLS 1024
#define SQ_STATIC_DEVICES 64
hipError_t sq_static_scratch(double** ptr);
// slot capacity of the variant that serves a need of kc slots per column
// (0: none)
int sq_kc_variant(bool fused, int kc);
int sq_img_limit(int nc);
int sq_gram_limit(int nc);
hipError_t sq_launch_reduce(const PlanDev& P, const int* cells, int ncells, int col0, int ncol,
                            hipStream_t s);
bool sq_nc_supported(int nc);
}
