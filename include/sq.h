/*
 * sq.h -- C ABI of the MI355X (gfx950) infinite-cell Clenshaw-Curtis
 * Spectral Quadrature (SQ) hot path.
 *
 * Operation (Sharma, Hamel, Bethkenhagen, Pask, Suryanarayana, arXiv
 * 2006.03697, Sec. IV and App. A): for every finite-difference node q of an
 * orthorhombic periodic cell, the nodal Hamiltonian H_q (the Hamiltonian
 * restricted to the cube of side 2 R_cut centred at q: 12th-order FD
 * Laplacian, local potential, atom-centred nonlocal projectors of every atom
 * image in R^3) is scaled to Hhat_q = (H_q - chi_q)/zeta_q from its extreme
 * eigenvalues; the Chebyshev three-term recurrence t^{j+1} = 2 Hhat t^j -
 * t^{j-1} from the unit vector w_q, weighted by the Clenshaw-Curtis
 * Fermi-Dirac coefficients c_q^j, gives the density-matrix column
 * d_q = sum' c_q^j t^j, from which the electron density
 * rho_q = (2/dV) sum' c_q^j rho_q^j, the band energy
 * 2 sum_q sum' (chi_q c_q^j + zeta_q d_q^j) rho_q^j, the kinetic and
 * nonlocal density-matrix stress, the pressure and the local
 * exchange-correlation stress term follow.
 *
 * Units: Hartree atomic units (Ha, Bohr).  All host-side scalars and arrays
 * are IEEE binary64 unless stated otherwise.
 *
 * Conventions: node i = ix + n0 (iy + n1 iz) at position h (ix, iy, iz);
 * Voigt order (11, 22, 33, 23, 13, 12); 3x3 blocks row-major (alpha, beta).
 *
 * Ownership: sq_setup copies every input, so the caller may free its
 * arrays on return.  The plan owns all device memory it allocates (through
 * the caller's allocator when one is given, else hipMalloc) and releases it
 * in sq_destroy.  Output buffers are owned by the caller.
 *
 * Errors: every entry point returns a status; nothing aborts across the
 * ABI.  On error the outputs are left untouched and sq_last_error() holds a
 * message.  A plan is used from one host thread at a time; separate plans
 * are independent.  Work is enqueued on the stream given at setup and every
 * call returns after that stream has finished the call's work.
 */
#ifndef SQ_H
#define SQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sq_plan_s* sq_plan;

typedef enum {
  SQ_OK = 0,
  SQ_E_ARG = 1,     /* invalid argument (shape, range, capacity)            */
  SQ_E_ALLOC = 2,   /* device allocation failed                              */
  SQ_E_DEVICE = 3,  /* HIP runtime error                                     */
  SQ_E_BOUNDS = 4,  /* a Chebyshev moment left [-1, 1]: spectral bounds bad  */
  SQ_E_NOCONV = 5,  /* Fermi level not bracketed / not found                 */
  SQ_E_STATE = 6    /* call order violated (e.g. stress before density)     */
} sq_status;

/* Working precision of the Chebyshev recurrence vectors (Sec. IV).  The
 * spectral-bound Lanczos, the moments' inner products, the coefficients, the
 * Fermi level and every reduction are FP64 in all modes.
 *
 * Moments: when every cell of the plan has max(K, ceil(npl / 2)) <= 63, the
 * plan runs that many FP64 Lanczos steps per node and takes the moments
 * rho_q^j, j <= npl, from the Lanczos tridiagonal (w^T p(H) w = e_1^T p(T) e_1
 * for degree <= 2k after k steps; the bounds use the first K steps only).
 * There is then no moments recurrence pass and the moments are FP64 in every
 * mode.  Otherwise a recurrence pass on the cube forms them, in the
 * precision below.
 *   SQ_FP64          FP64 vectors in both passes.
 *   SQ_MIXED         FP32 vectors in the moments pass and in the stress pass.
 *   SQ_MIXED_STRESS  FP64 vectors in the moments pass (so mu, rho and the
 *                    band energy are those of SQ_FP64), FP32 vectors in the
 *                    stress pass.  For cells whose Fermi level is
 *                    ill-conditioned (low density of states at mu) the FP32
 *                    moments of SQ_MIXED shift mu and through it the stress;
 *                    this mode avoids that at the cost of the FP64 moments. */
typedef enum { SQ_FP64 = 0, SQ_MIXED = 1, SQ_MIXED_STRESS = 2 } sq_precision;
typedef enum { SQ_MU_SOLVE = 0, SQ_MU_FIXED = 1 } sq_mu_mode;

/* One analytic species (the paper's pseudopotential data, Sec. V.A, is
 * replaced by Gaussians): V(r) = -v_amp exp(-r^2 / (2 v_sigma^2)) for
 * r < v_rcut; one s projector p(r) = exp(-r^2 / (2 p_sigma^2)) for
 * r < p_rcut with energy gamma; z_val valence electrons. */
typedef struct {
  double v_amp, v_sigma, v_rcut;
  double p_sigma, p_rcut, gamma;
  double z_val;
} sq_species;

/* One periodic orthorhombic cell (Sec. II: sides L, nuclei R, N_e). */
typedef struct {
  double L[3];          /* cell sides; L[a] / h must be an integer (1e-9)   */
  double h;             /* mesh size                                         */
  int fd_half_order;    /* M: FD order 2M; 6 (12th order, Sec. V) supported */
  int n_atoms;
  const double* pos;    /* [n_atoms][3] positions, wrapped into [0, L)      */
  const int* species;   /* [n_atoms] index into sp                          */
  int n_species;
  const sq_species* sp; /* [n_species]                                      */
  double n_electrons;   /* N_e; < 0 means the sum of z_val                  */
  double rcut;          /* truncation radius: cube of (2 floor(rcut/h)+1)^3 */
  int npl;              /* Chebyshev degree n_pl (>= 1)                     */
  double kT;            /* smearing sigma (Fermi-Dirac), Ha, > 0            */
  int mu_mode;          /* sq_mu_mode                                       */
  double mu;            /* Fermi level used when mu_mode == SQ_MU_FIXED      */
  int lanczos_steps;    /* K of the spectral-bound Lanczos (>= 2; 0 -> 20)  */
} sq_cell;

/* Plan options.  A zero-initialised struct gives the defaults.
 *   precision          sq_precision.
 *   hip_stream         hipStream_t the plan's work is ordered on (NULL: the
 *                      default stream).
 *   dev_alloc/dev_free device memory for the plan (NULL: hipMalloc/hipFree).
 *   outputs_on_device  1: the output pointers of the calls below are device
 *                      pointers.
 *   use_graph          1: sq_density and the stress pass capture their launch
 *                      sequence in a HIP graph on a private stream at their
 *                      first call for a given cell selection, and replay the
 *                      graph on hip_stream afterwards (the host only reads
 *                      back the Fermi level, the error flags and the sums).
 *   autotune           1: at set-up, time the kernel variants of every
 *                      node group (slot capacity 16 or 24 with the projector
 *                      weights of plane 0 in registers, or 48 recomputing
 *                      them; persistent or one-workgroup-per-node launch) on
 *                      a sample of its nodes and keep the fastest per kernel;
 *                      0: the smallest capacity and `persistent` below.
 *   tune_cache         path of a JSON file of tuned choices: read at set-up
 *                      (a hit skips the timing), rewritten after tuning;
 *                      NULL: none.  Keys name the device, cube width, slot
 *                      needs, precision and kernel.
 *   cheb_quad_points   M_q of the Gauss-Chebyshev rule for the coefficient
 *                      integrals of Sec. IV (a power of two >= 4 (n_pl + 2));
 *                      0: the smallest power of two >= max(4 (n_pl + 2),
 *                      8 zeta_q / kT) per node.
 *   persistent         0: one workgroup per node; 1: a persistent grid that
 *                      takes nodes from an atomic work counter (for groups
 *                      whose columns need at most 16 projector slots).
 *   inject             0 in normal use.  Bits of sq_inject force the error
 *                      paths for tests, from the host, with every kernel
 *                      running to its normal end: SQ_INJECT_NARROW halves
 *                      every node's spectral interval about its centre, so
 *                      that the Chebyshev moments leave [-1, 1] and
 *                      sq_density returns SQ_E_BOUNDS; SQ_INJECT_MU_CAP
 *                      stops the Fermi-level search after 2 updates, so that
 *                      sq_density returns SQ_E_NOCONV.  Other bits:
 *                      SQ_E_ARG.
 * Node columns of a launch are ordered by decreasing Chebyshev degree
 * (longest first). */
typedef struct {
  int precision;
  void* hip_stream;
  void* (*dev_alloc)(size_t bytes, void* ctx);
  void (*dev_free)(void* ptr, void* ctx);
  void* alloc_ctx;
  int outputs_on_device;
  int use_graph;
  int autotune;
  const char* tune_cache;
  int cheb_quad_points;
  int persistent;
  int inject;
} sq_options;

typedef enum { SQ_INJECT_NARROW = 1, SQ_INJECT_MU_CAP = 2 } sq_inject;

/* Validate the cells, build the per-cell tables (grid, atom images, local
 * potential, per-tile image lists, the Gram matrix of each node's projectors)
 * and allocate the plan's device memory (about 13.5 KB per node plus
 * 16 (n_pl + 2) bytes per node: 12 KB of it the Gram matrix).
 * Sec. IV: grid K_Omega, cube of side 2 R_cut, atoms of R^3 whose projectors
 * meet the cube.  Returns SQ_E_ARG for a non-integral L/h, R_cut < h,
 * npl outside [1, 256], kT <= 0, an FD order other than 12, or a cube
 * narrower than 7 or wider than 25 nodes. */
sq_status sq_setup(const sq_cell* cells, int n_cells, const sq_options* opt, sq_plan* out);

/* Spectral bounds, Chebyshev moments, Fermi level and density (Sec. IV).
 * cell = -1 runs every cell of the plan in the same launches.
 * rho: [N_d] per cell (concatenated in cell order), may be NULL;
 * mu: one per cell, may be NULL.  The Fermi level is searched entirely on
 * the device within a fixed budget of evaluations; the host synchronises
 * once, at the end.  SQ_E_BOUNDS if a moment left [-1, 1] (tolerance 1e-6
 * with FP64 moments, 1e-4 with FP32 ones), SQ_E_NOCONV if N_e is not
 * bracketed or |N - N_e| <= 1e-13 N_e was not reached. */
sq_status sq_density(sq_plan plan, int cell, double* rho, double* mu);

/* Band energy 2 sum_q sum'_j (chi_q c_q^j + zeta_q d_q^j) rho_q^j (App. A),
 * one value per cell.  Needs sq_density first (SQ_E_STATE otherwise). */
sq_status sq_energy(sq_plan plan, int cell, double* e_band);

/* Kinetic + nonlocal density-matrix stress (Sec. IV) divided by |Omega|:
 * sigma_voigt [6] per cell; parts [18] per cell (nullable): the node sums
 * of K (3x3) then N (3x3), not divided by |Omega|.  Needs sq_density. */
sq_status sq_stress(sq_plan plan, int cell, double* sigma_voigt, double* parts);

/* For callers that cannot allocate device memory at call time (code under
 * HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): sq_stress with the per-cell sums of its stress reduction
 * formed in a static device array of the library instead of plan memory.
 * Same arguments, outputs (bit for bit) and errors as sq_stress; it
 * allocates no device memory (no hipMalloc, no allocator callback) and, on
 * success, no host memory, and always runs the stress pass eagerly, never
 * from a captured graph.  The array holds 1024 rows of 28 doubles (229 KB); each
 * GPU the library runs on holds its own copy until the process ends, and
 * its address is taken once per device at sq_setup.  SQ_E_ARG for a plan
 * of more than 1024 cells.  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (several host threads or streams) race.
 * The plan's own stress sums are not written, so sq_pressure after it runs
 * its own stress pass unless sq_stress has run since the last
 * sq_density. */
sq_status sq_stress_static(sq_plan plan, int cell, double* sigma_voigt, double* parts);

/* Pressure, P = -(sigma_11 + sigma_22 + sigma_33)/3 of the kinetic + nonlocal
 * stress, one value per cell in each output (either may be NULL), in two
 * forms:
 *   p_direct  the direct form of App. A: the kinetic trace is taken from the
 *             band energy, -2 E_band + 2 sum_q dV V_q rho_q + 2 E_nl (the
 *             Chebyshev expansion of H times the density matrix), so no
 *             second derivative of the density matrix enters; the nonlocal
 *             part is tr N.  P = -(that + tr N) / (3 |Omega|), with
 *             E_nl = 2 sum_q sum_I gamma dV chi_I(x_q) chi_I^T d_q.
 *   p_trace   -tr(K + N) / (3 |Omega|) from the stress of sq_stress.
 * The two agree to the discretisation and truncation error (the 12th-order
 * Laplacian is not the square of the 12th-order gradient, and the expansion
 * of x g(x) stops at degree n_pl).  Runs the stress pass first when
 * sq_stress has not run since the last sq_density; needs sq_density
 * (SQ_E_STATE otherwise). */
sq_status sq_pressure(sq_plan plan, int cell, double* p_direct, double* p_trace);

/* Exchange-correlation energy E_xc = sum_q dV rho_q eps_xc(rho_q) and the
 * exchange-correlation stress term of Sec. II for a local functional,
 * delta_ab (E_xc - sum_q dV rho_q v_xc(rho_q)) / |Omega| (isotropic: one
 * value per cell, the diagonal), from the SQ density.  LDA: Slater exchange
 * and the Perdew-Wang 1992 correlation of the unpolarised electron gas;
 * nodes with rho_q <= 0 contribute nothing.  Either output may be NULL.
 * Needs sq_density (SQ_E_STATE otherwise). */
sq_status sq_xc(sq_plan plan, int cell, double* e_xc, double* sigma_xc);

/* Per-node records for a list of nodes of one cell (the per-node terms of
 * the SQ sums of Sec. IV: the density rho_q = (2/dV) sum' c_q^j rho_q^j, the
 * node's share of the kinetic and nonlocal stress, and App. A's energy
 * terms): out [n][24] =
 * rho_q, band-energy density e_q, K (9), N (9), nonlocal energy density
 * 2 sum_I gamma dV chi_I(x_q) chi_I^T d_q, local-potential energy
 * dV V_q rho_q, exchange-correlation energy dV rho_q eps_xc and stress
 * density dV rho_q (eps_xc - v_xc).  K, N and the nonlocal energy need the
 * stress pass after the last sq_density (zeros otherwise).  nodes are host
 * arrays. */
sq_status sq_nodes(sq_plan plan, int cell, const int64_t* nodes, int64_t n, double* out);

/* Per-node spectral bounds lambda_lo, lambda_hi ([N_d] each, host arrays;
 * either may be NULL): the interval taken for the extreme eigenvalues
 * lambda_q^min, lambda_q^max of the nodal Hamiltonian H_q that give
 * chi_q and zeta_q of Sec. IV (K-step Lanczos from w_q, the extreme Ritz
 * values widened by their residuals).  sq_moments: the Chebyshev moments
 * rho_q^j = w_q^T t_q^j of Sec. IV for a list of nodes (out [n][npl+1]).
 * Both need sq_density (SQ_E_STATE otherwise); SQ_E_ARG for a node index
 * outside [0, N_d). */
sq_status sq_bounds(sq_plan plan, int cell, double* lam_lo, double* lam_hi);
sq_status sq_moments(sq_plan plan, int cell, const int64_t* nodes, int64_t n, double* out);

/* Lanczos tridiagonals behind the spectral bounds, for a list of nodes:
 * out [n][2K+1] = steps taken, alpha_1..alpha_K, beta_1..beta_K (zeros past
 * the steps taken), K = the cell's lanczos_steps.  Needs sq_density. */
sq_status sq_lanczos(sq_plan plan, int cell, const int64_t* nodes, int64_t n, double* out);

/* Plan queries (info has 14 entries): info[0] = N_d, info[1] = n_c,
 * info[2] = npl, info[3] = number of atom images, info[4] = max images in a
 * node tile, info[5..7] = largest number of images reaching one cube,
 * crossing one cube column, and nonzero at one node, info[8] = number of
 * (node, projector) pairs over all nodes' cubes (measured at set-up),
 * info[9] = the Lanczos step count K in effect (lanczos_steps, 0 -> 20),
 * info[10] = stored Gram-matrix entries over the cell's nodes (each read
 * at every recurrence step of its node: 12 bytes per entry), info[11] =
 * nodes whose Gram matrix is stored (one projector sweep per step; the
 * others take two), info[12] = Lanczos steps run per node (K, or
 * ceil(npl / 2) when more and the moments come from the tridiagonal),
 * info[13] = 1 when the moments come from the Lanczos tridiagonal, 0 when
 * from the recurrence pass. */
sq_status sq_cell_info(sq_plan plan, int cell, int64_t* info);

/* Device time of each phase accumulated over the calls since the last reset
 * (HIP events on the plan's stream), ms [7] and call counts [7] in the
 * order: Lanczos bounds, bound extraction, Chebyshev moments, Fermi level,
 * coefficients + density, stress pass, final reductions.  reset != 0 zeroes
 * the accumulators after reading.  Either output may be NULL. */
sq_status sq_phase_times(sq_plan plan, int reset, double* ms, int64_t* count);

const char* sq_status_str(sq_status s);
/* Message of the last failed call on the plan; with plan == NULL, of the
 * last failed sq_setup on the calling thread. */
const char* sq_last_error(sq_plan plan);
void sq_destroy(sq_plan plan);

#ifdef __cplusplus
}
#endif

#endif /* SQ_H */
