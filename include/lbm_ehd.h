/*
 * lbm_ehd.h -- C ABI of the MI355X (gfx950) implementation of the
 * phase-field multiple-relaxation-time lattice Boltzmann method for two-phase
 * electrohydrodynamic flow driven by the Onsager-Wien effect
 * (Zheng, Wang, Xiong, Huang, Luo, arXiv 2501.04920, Sec. 4).
 *
 * One time step advances five coupled lattice Boltzmann equations on a 2-D
 * grid (lattice units, dx = dt = 1):
 *   f  (D2Q9)  incompressible Navier-Stokes, Eq. (51)-(57)
 *   h  (D2Q9)  conservative Allen-Cahn phase field, Eq. (27)-(33)
 *   p  (D2Q5)  cations, Eq. (34)-(43)
 *   n  (D2Q5)  anions, Eq. (35)-(43)
 *   g  (D2Q5)  electric potential, Eq. (44)-(49)
 * coupled through the isotropic finite differences of Eq. (59), the
 * phase-interpolated properties of Eq. (61), the field-enhanced dissociation
 * and recombination source of Eq. (5)-(6) and the surface-tension and
 * electric forces of Eq. (12)-(14).
 *
 * Geometry: x is periodic; the anode (psi = dpsi) lies half a lattice spacing
 * below row 0 and the cathode (psi = 0) half a spacing above row ny-1
 * (boundary conditions of Eq. (64) and Sec. 5.1).
 *
 * Conventions for every function:
 *   - the return value is LBM_OK (0) or a negative LBM_E* code; on error
 *     lbm_ehd_last_error() returns a message for the calling thread;
 *   - host pointers are caller-owned and only read/written during the call;
 *   - device pointers are hipMalloc'd (or PyTorch-allocated) memory on the
 *     device the handle was created on;
 *   - functions that enqueue GPU work do so on the handle's stream and return
 *     without waiting, unless they are documented to synchronise.
 * A handle is not thread-safe; distinct handles may be used concurrently.
 */
#ifndef LBM_EHD_H
#define LBM_EHD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#ifndef LBM_API
#define LBM_API __attribute__((visibility("default")))
#endif

typedef int32_t lbm_status;
#define LBM_OK 0
#define LBM_EINVAL (-1)     /* invalid argument or parameter set */
#define LBM_ENOMEM (-2)     /* device or host allocation failed */
#define LBM_EDEVICE (-3)    /* a HIP call failed */
#define LBM_ENONFINITE (-4) /* the state contains NaN or Inf */
#define LBM_ESTATE (-5)     /* call out of order (e.g. step before init) */
#define LBM_ERANGE (-6)     /* caller buffer too small */

/* Storage and arithmetic precision.  Populations are always stored as
 * deviations from a reference state (h: w_i/2, p and n: wbar_i c0, g: the
 * equilibrium of the uncharged linear potential, f: 0; 16-bit storage adds
 * node-local references).  The rest populations that carry the conserved
 * contents (h0; with 16-bit storage also p0 and n0) take what a node's
 * stored moving populations leave of its content, so that each collision
 * conserves phi and the ion contents: they are FP64 (conserved to FP64
 * rounding) except h0 with FP32 storage, a 32-bit fixed-point value
 * (2^-30 units) booked in integers against the fixed-point images of the
 * moving populations, which conserves the sum of phi over the grid
 * exactly. */
#define LBM_FP64 0       /* FP64 storage, FP64 arithmetic */
#define LBM_FP32 1       /* FP32 storage.  Arithmetic: FP64 for the phase
                            ring and its stencils, the macroscopic quantities
                            and all five collisions; the FP64 results are
                            rounded once, to FP32, when stored.  (phi u)(t-1)
                            is kept in FP32. */
#define LBM_FP16_STORE 2 /* binary16 storage, FP32 arithmetic */
#define LBM_BF16_STORE 3 /* bfloat16 storage, FP32 arithmetic */
#define LBM_FP32_F64 5   /* FP32 storage, FP64 arithmetic throughout, and
                            (phi u)(t-1) in FP64 */

/* Boundary conditions in y. */
#define LBM_ELECTRODES 0 /* Eq. (64a): anode/cathode with ion conditions of Sec. 5.1 */
#define LBM_INSULATING 1 /* electrodes for psi, f, h; ions bounce back (no ion flux) */
#define LBM_PERIODIC 2   /* periodic in y as well (no walls) */

/* Field selection bits for lbm_ehd_get_fields(). */
#define LBM_FIELD_PHI (1u << 0)   /* order parameter, Eq. (33) */
#define LBM_FIELD_PSI (1u << 1)   /* potential, Eq. (49) */
#define LBM_FIELD_CP (1u << 2)    /* cation concentration c+, Eq. (42) */
#define LBM_FIELD_CM (1u << 3)    /* anion concentration c-, Eq. (42) */
#define LBM_FIELD_RHOE (1u << 4)  /* free charge density, Eq. (8) */
#define LBM_FIELD_UX (1u << 5)    /* velocity, Eq. (56) */
#define LBM_FIELD_UY (1u << 6)
#define LBM_FIELD_P (1u << 7)     /* hydrodynamic pressure, Eq. (57) */
#define LBM_FIELD_EX (1u << 8)    /* electric field E = -grad psi, Eq. (9), (59) */
#define LBM_FIELD_EY (1u << 9)
#define LBM_FIELD_ALL 0x3FFu

/*
 * Simulation parameters in lattice units.  Properties of the two phases are
 * given for the outer ("v") phase plus the ratio liquid/vapour of Eq. (60);
 * every property is interpolated linearly in phi (Eq. 61).
 */
typedef struct {
  int32_t nx, ny;          /* grid; nx >= 2, 2 <= ny <= 65536 (one row of workgroups
                              per lattice row in the helper kernels), and a
                              population buffer below 4 GiB (32-bit byte offsets:
                              lines x (ny + 2) x pitch x element size, pitch = nx
                              rounded up to 64); LBM_EINVAL otherwise */
  int32_t precision;       /* LBM_FP64, LBM_FP32, LBM_FP16_STORE, LBM_BF16_STORE,
                              LBM_FP32_F64 */
  int32_t walls;           /* LBM_ELECTRODES, LBM_INSULATING, LBM_PERIODIC */
  int32_t reaction;        /* 1: R of Eq. (5)-(6); 0: R = 0 (leaky-dielectric limit, Sec. 5.2) */
  int32_t poisson_form;    /* 1: source (rho_e + grad eps . grad psi)/eps, whose steady
                              state is div(eps grad psi) = -rho_e (Eq. 7);
                              0: rho_e/eps as printed in Eq. (44) */
  int32_t poisson_norm;    /* 1: source weights w_i/(1 - w_0) so that the steady state
                              solves Eq. (7); 0: weights w_i as printed in Eq. (44) */
  int32_t flow;            /* 1: solve Eq. (51); 0: u = 0 and f is left as it is */
  int32_t ion_force;       /* 1: keep L_i of Eq. (39); 0: drop it */
  int32_t poisson_iters;   /* extra g-only sweeps before every step (0 = one fused
                              g update per step) */
  int32_t mask_f, mask_h, mask_p, mask_n, mask_g; /* bit k set: MRT row k relaxes with
                              1/tau (Eq. 30, 37, 47, 55); other rows relax with s_free */
  int32_t side_walls;      /* 0: periodic in x; 1: the other boundaries of Eq. (64),
                              walls halfway at x = -1/2 and x = nx - 1/2 with u = 0
                              (f bounces back), zero normal derivative of c+, c-
                              and psi (ion and potential populations bounce back,
                              zero flux) and of phi (h reflects specularly, a
                              neutral wall; bounce-back at the corners); the
                              stencils see the wall column mirrored */
  int32_t local_field;     /* 0: E = -grad psi by the stencil of Eq. (59);
                              1: E = sum_i c_i g_i / (c_s^2 tau_g) from the node's
                              incoming g (Eq. 50), and grad psi = -E wherever it
                              enters (forces, reaction, ion drift, Poisson source) */
  int32_t poisson_max;     /* with poisson_tol > 0: at most this many g-only sweeps
                              per step */
  double rho_v, rho_r;     /* density, outer phase; ratio (Eq. 60) */
  double eta_v, eta_r;     /* dynamic viscosity; tau_f = 1/2 + eta/(rho c_s^2), Eq. (55) */
  double M_phi;            /* phase-field mobility; tau_h = 1/2 + M_phi/c_s^2, Eq. (30) */
  double W;                /* interface width, Eq. (2) */
  double zeta;             /* surface tension; beta = 12 zeta/W, kappa = 3 zeta W/2 (Eq. 13) */
  double theta;            /* artificial diffusion of the Poisson LBE; tau_g = 1/2 + theta/c_s^2 */
  double dpsi;             /* anode potential psi_0 (cathode psi_1 = 0) */
  double eps_v, eps_r;     /* permittivity; ratio */
  double mu_v, mu_r;       /* cation mobility, outer phase; ratio */
  double m_ratio;          /* m = mu_- / mu_+ (Eq. 23) */
  double v_th;             /* k_B T_r / e_0: D = v_th mu (Sec. 2.2); tau = 1/2 + D/c_s^2 (Eq. 37) */
  double c0;               /* zero-field concentration (Eq. 5) */
  double q;                /* elementary charge e_0: rho_e = q (c+ - c-), delta = q (mu+ + mu-)/eps */
  double gamma_v;          /* Onsager constant of Eq. (6) in the outer phase; gamma ~ 1/eps */
  double force_x, force_y; /* external body-force density added to F (tests) */
  double s_free;           /* rate of the MRT rows not in the masks (1.0 in Sec. 6) */
  double poisson_tol;      /* > 0: converged-Poisson mode.  Before every step, g-only
                              sweeps in groups of poisson_iters (>= 1) until the
                              convergence residual of lbm_ehd_presolve_to falls below
                              poisson_tol, or poisson_max sweeps (each check
                              synchronises the stream); 0: poisson_iters fixed sweeps */
  double n_eps;            /* the unit normal grad(phi)/|grad(phi)| of Eq. (1), (32) is
                              evaluated as grad(phi)/sqrt(|grad(phi)|^2 + n_eps^2)
                              (default 1e-4): the bare form is undefined where
                              grad(phi) = 0 and lambda is not small (a droplet's centre),
                              and there it turns rounding into O(1e-5) changes of phi.
                              0: bare form, taken as 0 where |grad(phi)| < 1e-12 */
  int32_t diag_every;      /* > 0: watchdog.  lbm_ehd_step and lbm_ehd_run check
                              the state whenever the step count reaches a multiple
                              of diag_every (the FP64 invariant sums and non-finite
                              count of lbm_ehd_diagnostics; each check
                              synchronises the stream) and return LBM_ENONFINITE
                              as soon as a cell is not finite.  0: no checks */
  int32_t inplace;         /* 0: two population buffers (pull streaming between them);
                              1: one buffer, in-place streaming in the AA pattern (the
                              populations of a node alternate between its own slots,
                              reversed, and its neighbours' slots, step by step; wall
                              rules written back into the node's own slots).  Halves
                              the population memory; FP64, FP32 and binary16 storage
                              (LBM_FP64, LBM_FP32, LBM_FP32_F64, LBM_FP16_STORE; binary16
                              keeps its node-local references of h and g in the node's
                              own rest slots and its ion rest populations in their
                              FP64 planes, as with two buffers; not LBM_BF16_STORE),
                              electrodes, insulating or
                              y-periodic walls, no side walls, no local field, no
                              converged-Poisson mode (lbm_ehd_presolve_to is not
                              available).  Each step adds a pre-pass that writes phi'
                              and psi' of the nodes at the edges of the sweep's tiles
                              (first and last row of each band, first and last
                              column of each strip) to two planes, from which the
                              sweep takes the stencils' halo (in place a neighbouring
                              workgroup may already have overwritten the populations
                              they are moments of). */
  int32_t ion_q9;          /* 0: the ion LBEs on D2Q5 (weights of Eq. (26), matrix N
                              of Eq. (46); 33 populations per node, the default);
                              1: on D2Q9 as Eq. (34)-(38) write them, with the
                              weights of Eq. (25) and the matrix M of Eq. (28) (8
                              more lines per lattice row, 344 instead of 280 bytes
                              per node update with FP32 storage).  FP64 and FP32
                              storage (LBM_FP64, LBM_FP32, LBM_FP32_F64), electrodes,
                              insulating or y-periodic walls, with or without side
                              walls (where the ions bounce back), no local field,
                              two buffers */
  int32_t reserved;        /* 0 */
} lbm_ehd_params;

/*
 * Dimensionless description of a droplet case (Eq. 15, 23, 24, 60), mapped
 * to lattice parameters by lbm_ehd_params_from_groups().
 */
typedef struct {
  int32_t n;               /* grid n x n; the electrode gap d is n lattice spacings */
  int32_t precision;
  double radius;           /* initial droplet radius, lattice units */
  double W;                /* interface width, lattice units (Cn = W/d) */
  double Ca_E;             /* electric capillary number eps dpsi^2 r / (zeta d^2) */
  double W0;               /* conduction number e0 c0 d^2 / (eps dpsi) */
  double beta;             /* sqrt(O W0), Eq. (24) */
  double eps_r, mu_r, rho_r, eta_r, m_ratio;
  double sigma_r;          /* conductivity ratio; only with reaction = 0 (leaky model),
                              where it sets mu_r (sigma ~ mu at uniform c0); 0 = unused */
  int32_t reaction;        /* as in lbm_ehd_params */
  int32_t reserved;
  /* lattice choices (0 selects the default in brackets) */
  double U;                /* ionic drift speed mu_bar dpsi / d [0.01] */
  double alpha;            /* diffusion number D / (mu_bar dpsi) [0.01] */
  double zeta;             /* [1e-3] */
  double M_phi;            /* [0.1] */
  double eta_v;            /* [0.1] */
  double eps_v;            /* [1.0] */
} lbm_ehd_groups;

/*
 * Caller-supplied device memory and stream.  pop[0] and pop[1] each hold
 * pop_bytes (>= the size lbm_ehd_required_bytes() returns) and aux holds
 * aux_bytes; the library ping-pongs between pop[0] and pop[1] (with
 * inplace = 1 it uses pop[0] alone, and pop[1] may be NULL).  The memory
 * stays owned by the caller and must outlive the handle.  stream is a
 * hipStream_t (NULL: the null stream).
 */
typedef struct {
  void *stream;
  void *pop[2];
  size_t pop_bytes;
  void *aux;
  size_t aux_bytes;
} lbm_ehd_device;

typedef struct {
  int64_t step;            /* time steps taken since the last init */
  double sum_phi;          /* FP64 sum of phi over the grid (Eq. 33) */
  double sum_rhoe;         /* FP64 sum of rho_e (Eq. 8) */
  double sum_p, sum_n;     /* FP64 sums of sum_i p_i and sum_i n_i */
  int64_t nonfinite;       /* number of cells whose moments are NaN or Inf */
  double D, L, H;          /* deformation factor of Eq. (63) and its lengths; the
                              length along the field (y) through the phi-weighted
                              centroid and across it, from the phi = 1/2 crossings
                              (NaN when no droplet is found) */
  int64_t presolve_iters;  /* g-only sweeps of the last pre-solve since init */
  double presolve_residual;/* its convergence residual (lbm_ehd_presolve_to; NaN
                              after lbm_ehd_presolve or none) */
} lbm_ehd_diag;

typedef struct lbm_ehd lbm_ehd; /* opaque handle */

/* Fill *out with the defaults: FP32, electrodes, reaction on, the Eq. (7)
 * Poisson form, rates as in Sec. 6 (free rows 1.0), theta = 0.3 (Sec. 4.2). */
LBM_API lbm_status lbm_ehd_params_default(lbm_ehd_params *out);

/* Map dimensionless groups to lattice parameters:
 *   dpsi = n sqrt(Ca_E zeta/(eps_v R)), mu_bar = U n/dpsi, D = alpha mu_bar dpsi,
 *   q = W0 eps_v dpsi/(c0 n^2) with c0 = 1, gamma_v = (beta^2/W0) n/dpsi.
 * LBM_EINVAL on a non-positive group or an unreachable relaxation time. */
LBM_API lbm_status lbm_ehd_params_from_groups(const lbm_ehd_groups *g, lbm_ehd_params *out);

/* Bytes needed for each population buffer and for the aux buffer. */
LBM_API lbm_status lbm_ehd_required_bytes(const lbm_ehd_params *p, size_t *pop_bytes,
                                  size_t *aux_bytes);

/* Device bytes one simulation needs at most when the library allocates its
 * state (dev = NULL): both population buffers, the aux buffer and the
 * library's scratch (moment and field planes for readback, allocated on first
 * use; sums; the sweep's tile list).  For admission control by HBM
 * footprint.  LBM_EINVAL as lbm_ehd_required_bytes. */
LBM_API lbm_status lbm_ehd_footprint_bytes(const lbm_ehd_params *p, size_t *bytes);

/* Create a simulation on the current HIP device.  dev may be NULL, in which
 * case the library allocates (and later frees) the buffers itself and uses
 * the null stream.  LBM_EINVAL: any tau <= 1/2, a non-finite coefficient,
 * nx or ny < 2, unknown precision or walls. */
LBM_API lbm_status lbm_ehd_create(const lbm_ehd_params *p, const lbm_ehd_device *dev, lbm_ehd **out);

/* Initial droplet: phi = 1/2 (1 + tanh(2 (R - r)/W)) around (xc, yc), fluid at
 * rest with p = 0, ions at c0 (1 + noise xi) with xi in [-1, 1) from SplitMix64
 * outputs 2k+1 (cations) and 2k+2 (anions) of cell k = y nx + x, psi linear
 * between the electrodes, every population at its equilibrium.  Resets the
 * step counter.  Enqueues work. */
LBM_API lbm_status lbm_ehd_init_droplet(lbm_ehd *h, double xc, double yc, double radius,
                                double noise, uint64_t seed);

/* Initial state from host fields [ny][nx] (FP64): equilibrium populations for
 * phi, c+, c-, psi and velocity (ux, uy may be NULL: at rest), p = 0,
 * (phi u)(t-1) = phi u.  Synchronises. */
LBM_API lbm_status lbm_ehd_init_fields(lbm_ehd *h, const double *phi, const double *cp,
                               const double *cm, const double *psi, const double *ux,
                               const double *uy);

/* `iters` g-only sweeps of Eq. (44) with phi and rho_e held fixed (Poisson
 * pre-solve).  Enqueues work. */
LBM_API lbm_status lbm_ehd_presolve(lbm_ehd *h, int32_t iters);

/* Poisson pre-solve to a tolerance: g-only sweeps as in lbm_ehd_presolve
 * until the convergence residual falls below `tol`, or `max_iters` sweeps.
 * The paper states no stopping rule (Sec. 4.2 fixes only theta).  The
 * residual is the FP64 relative change of the potential over one sweep,
 * ||psi_{k+1} - psi_k||_2 / ||psi_{k+1}||_2, divided by the per-sweep decay
 * rate of the slowest mode of the Poisson LBE, pi^2 theta / ny^2 (a
 * diffusion with coefficient theta between electrodes ny apart), so that it
 * estimates the remaining relative error of psi.  It is formed from FP64
 * per-row sums in a fixed order (the same on every run) every
 * `check_every` sweeps.  *iters (sweeps done) and *residual (last residual)
 * may be NULL; both are also reported by lbm_ehd_diagnostics.  Synchronises
 * at each check.  LBM_EINVAL unless tol > 0, max_iters >= 1 and
 * check_every >= 1; LBM_ESTATE before init; LBM_ENONFINITE if the potential
 * is not finite. */
LBM_API lbm_status lbm_ehd_presolve_to(lbm_ehd *h, double tol, int32_t max_iters,
                                       int32_t check_every, int32_t *iters, double *residual);

/* One time step (poisson_iters extra g sweeps, or with poisson_tol > 0 g sweeps
 * to that tolerance, whose count and residual the diagnostics report as those
 * of the last pre-solve; then the fused sweep of all five equations).
 * Enqueues work (the watchdog of diag_every synchronises at its checks).
 * LBM_ESTATE before init or for a member of a batch; LBM_ENONFINITE from the
 * watchdog. */
LBM_API lbm_status lbm_ehd_step(lbm_ehd *h);

/* nsteps time steps, as many lbm_ehd_step calls.  With poisson_iters = 0 and
 * poisson_tol = 0, whole blocks of 16 steps are replayed from a HIP graph
 * captured at the first such block (one graph per parity of the current
 * buffer; dropped by lbm_ehd_set_launch), bitwise the same as launching the
 * steps one by one.  Enqueues work; errors as lbm_ehd_step. */
LBM_API lbm_status lbm_ehd_run(lbm_ehd *h, int64_t nsteps);

/* Macroscopic fields at the current time, FP64, layout [field][ny][nx] for
 * the selected bits of `mask` in increasing bit order.  n_doubles is the
 * capacity of `out`; LBM_ERANGE if it is too small.  Synchronises. */
LBM_API lbm_status lbm_ehd_get_fields(lbm_ehd *h, uint32_t mask, double *out, size_t n_doubles);

/* FP64 invariants (sums in a fixed order, independent of launch shape), the
 * non-finite count and the deformation factor.  Synchronises.  Returns
 * LBM_ENONFINITE (after filling *out) if any cell is not finite. */
LBM_API lbm_status lbm_ehd_diagnostics(lbm_ehd *h, lbm_ehd_diag *out);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): lbm_ehd_diagnostics without the
 * deformation factor, allocating nothing.  Fills step, sum_phi, sum_rhoe,
 * sum_p, sum_n, nonfinite and the pre-solve fields exactly as
 * lbm_ehd_diagnostics does (the same kernels and summation order), and sets
 * D, L and H to NaN.  The per-row partial sums live in a static device
 * array of the library, one per GPU, for grids of up to 16384 rows (0.9 MB,
 * held until the process ends); it keeps the last call's contents, and
 * calls that overlap on one GPU (from several threads or streams) race on
 * it.  No hipMalloc, hipFree or allocating library call is made.
 * Synchronises.  LBM_ERANGE if ny > 16384; LBM_ESTATE before init;
 * LBM_ENONFINITE (after filling *out) if any cell is not finite. */
LBM_API lbm_status lbm_ehd_invariants_noalloc(lbm_ehd *h, lbm_ehd_diag *out);

/* Current step count. */
LBM_API int64_t lbm_ehd_time(const lbm_ehd *h);

/*
 * Checkpoint and resume.  The state of a simulation (its current population
 * buffer, the aux buffer with (phi u)(t-1) and the rest populations,
 * the step count) fits in *bytes of host memory.  lbm_ehd_save_state copies
 * it out (synchronises); lbm_ehd_load_state copies a saved state into a
 * simulation created with the same grid and storage precision and makes it
 * current.  The populations are stored as deviations from references that
 * depend on some parameters: the wall types (walls, side_walls), dpsi, c0,
 * the offset of the g references (theta, mask_g, s_free) and, with 16-bit
 * storage, the ion line offsets (c0, gamma_v, mu_v, m_ratio, reaction) and
 * the binary16 scales.  The saved state records them, and a load into a
 * simulation whose references differ is refused (LBM_EINVAL): the same bytes
 * would stand for another physical state.  Other parameters may differ; with
 * all parameters equal the simulation continues bitwise as the saved one
 * would have.  The buffer is caller-owned.  LBM_ESTATE for a member of a
 * batch (remove it first) or when saving before init; LBM_EINVAL on a NULL
 * argument or a state of another grid, precision, layout or references;
 * LBM_ERANGE if the buffer is too small.
 */
LBM_API lbm_status lbm_ehd_state_bytes(const lbm_ehd *h, size_t *bytes);
LBM_API lbm_status lbm_ehd_save_state(lbm_ehd *h, void *buffer, size_t bytes);
LBM_API lbm_status lbm_ehd_load_state(lbm_ehd *h, const void *buffer, size_t bytes);

/* Launch shape of the fused sweep: `waves` wavefronts per workgroup (1, 2, 4
 * or 8; a workgroup owns a strip of 64 * waves columns and walks down a band of
 * `tile_rows` rows, tile_rows >= 1, clamped to ny).  Results do not depend on
 * the shape (every node runs the same arithmetic), only the speed does.
 * lbm_ehd_create picks a default from the grid size; the shape applies from
 * the next step.  LBM_EINVAL on other values. */
LBM_API lbm_status lbm_ehd_set_launch(lbm_ehd *h, int32_t waves, int32_t tile_rows);
LBM_API lbm_status lbm_ehd_get_launch(const lbm_ehd *h, int32_t *waves, int32_t *tile_rows);

/*
 * Batched sweeps.  Several initialised simulations of any grid sizes, with
 * the same storage precision, poisson_iters = 0 and poisson_tol = 0, are
 * advanced together: each step is ONE kernel launch over the tiles of all
 * members (each tile runs the single-simulation tile code on its own
 * member), and whole blocks of steps are captured once in a HIP graph and
 * replayed.  The sweep has three compiled forms (plain; with side walls;
 * with side walls and the local field); members of different forms are
 * launched separately, one launch per form present.  Every member's
 * arithmetic is the same as when it steps alone, so its results are bitwise
 * those of lbm_ehd_run.
 *
 * The batch keeps pointers to its members (lbm_ehd_destroy of a member
 * removes it from its batch first).  A simulation belongs to at most one
 * batch.  While in a batch, members are stepped on the batch's stream only:
 * lbm_ehd_step, lbm_ehd_run, lbm_ehd_presolve, lbm_ehd_presolve_to,
 * lbm_ehd_init_droplet, lbm_ehd_init_fields, lbm_ehd_load_state and
 * lbm_ehd_set_launch return LBM_ESTATE for a member.  Their step counters
 * and current buffers are kept up to date, so lbm_ehd_get_fields,
 * lbm_ehd_diagnostics and lbm_ehd_save_state work on them after
 * lbm_ehd_batch_synchronize.
 */
typedef struct lbm_ehd_batch lbm_ehd_batch;

/* Group `n` members (n >= 0; NULL list allowed for n = 0) on `stream`, which
 * must not be the legacy default stream (graphs cannot be captured there);
 * NULL: the batch creates its own blocking stream of default priority,
 * ordered with the default stream and destroyed with the batch.  LBM_EINVAL on mixed precisions, members with
 * poisson_iters != 0 or poisson_tol > 0, duplicates or members on another device; LBM_ESTATE if
 * a member is not initialised. */
LBM_API lbm_status lbm_ehd_batch_create(lbm_ehd *const *sims, int32_t n, void *stream,
                                        lbm_ehd_batch **out);
/* Add a member (same checks as create; the member's own stream is
 * synchronised first) or remove one (the batch stream is synchronised, so
 * the removed member's state is complete).  Takes effect at the next run. */
LBM_API lbm_status lbm_ehd_batch_add(lbm_ehd_batch *b, lbm_ehd *h);
LBM_API lbm_status lbm_ehd_batch_remove(lbm_ehd_batch *b, lbm_ehd *h);
/* Number of members, -1 for NULL. */
LBM_API int32_t lbm_ehd_batch_size(const lbm_ehd_batch *b);
/* Launch shape of the batched sweep (as lbm_ehd_set_launch; one shape for
 * all members; bands are clamped to each member's ny). */
LBM_API lbm_status lbm_ehd_batch_set_launch(lbm_ehd_batch *b, int32_t waves, int32_t tile_rows);
LBM_API lbm_status lbm_ehd_batch_get_launch(const lbm_ehd_batch *b, int32_t *waves,
                                            int32_t *tile_rows);
/* Steps per captured graph block (even, default 16; 0: no graphs). */
LBM_API lbm_status lbm_ehd_batch_set_graph_steps(lbm_ehd_batch *b, int32_t steps);
/* Advance every member by `nsteps` (whole blocks by graph replay, the rest
 * by direct launches).  Asynchronous on the batch stream. */
LBM_API lbm_status lbm_ehd_batch_run(lbm_ehd_batch *b, int64_t nsteps);
/* Choose the launch shape: time `steps_per_trial` (even, >= 2) steps of the
 * batch for each candidate (waves 1, 2, 4, 8 not much wider than the widest
 * member x bands of 2, 4, 8, 16, 32 rows) with HIP events and keep the
 * fastest.  The trial steps are real steps of every member (results do not
 * depend on the shape); their count is returned in *steps_taken.  Blocks
 * until the trials are done. */
LBM_API lbm_status lbm_ehd_batch_autotune(lbm_ehd_batch *b, int32_t steps_per_trial,
                                          int32_t *waves, int32_t *tile_rows,
                                          int64_t *steps_taken);
/* Wait for the batch's work.  LBM_EDEVICE if a kernel failed. */
LBM_API lbm_status lbm_ehd_batch_synchronize(lbm_ehd_batch *b);
/* Release the batch (not its members).  NULL is allowed. */
LBM_API lbm_status lbm_ehd_batch_destroy(lbm_ehd_batch *b);

/*
 * Serving: a request server with continuous batching.  Each request is a
 * droplet simulation (parameters, droplet, number of steps).  Requests wait
 * in arrival order; at every scheduling round the server retires finished
 * requests, admits waiting ones that fit the HBM budget (first fit in
 * arrival order, by lbm_ehd_footprint_bytes), and advances all running
 * requests by one block of steps as members of one batch (one sweep launch
 * per step).  State stays resident on the device from admission to release.
 * A request's results are bitwise those of the same simulation run alone.
 * Single-threaded: call the server functions from one thread.  Errors of the
 * server functions are described by lbm_ehd_server_last_error().
 */
typedef struct lbm_ehd_server lbm_ehd_server;

enum { LBM_REQ_QUEUED = 0, LBM_REQ_RUNNING = 1, LBM_REQ_DONE = 2, LBM_REQ_FAILED = 3 };

typedef struct {
  int64_t id;
  int32_t state;           /* LBM_REQ_* */
  int32_t reserved;
  int64_t steps_done, steps_total;
  double t_submit, t_start, t_done; /* seconds since server creation; -1 if not yet */
  size_t footprint;        /* device bytes counted against the budget */
  lbm_ehd_diag diag;       /* at completion (D, sums) */
} lbm_ehd_request_info;

/* A server with `hbm_budget_bytes` of device memory for request state and
 * blocks of at most `block_steps` steps (even, >= 2) between scheduling
 * rounds.  Runs on its own stream on the current device. */
LBM_API lbm_status lbm_ehd_server_create(size_t hbm_budget_bytes, int32_t block_steps,
                                         lbm_ehd_server **out);
/* Queue a request: parameters (poisson_iters = 0; one storage precision per
 * server), droplet as lbm_ehd_init_droplet, `nsteps` steps.  The id is
 * written to *id.  LBM_ERANGE if the request alone exceeds the budget. */
LBM_API lbm_status lbm_ehd_server_submit(lbm_ehd_server *s, const lbm_ehd_params *p, double xc,
                                         double yc, double radius, double noise, uint64_t seed,
                                         int64_t nsteps, int64_t *id);
/* One scheduling round: retire, admit, launch the next block (asynchronous;
 * retiring waits for the blocks before it).  Writes the numbers of running
 * and queued requests (either pointer may be NULL). */
LBM_API lbm_status lbm_ehd_server_advance(lbm_ehd_server *s, int32_t *running, int32_t *queued);
/* State, timestamps and (when done) diagnostics of a request. */
LBM_API lbm_status lbm_ehd_server_info(lbm_ehd_server *s, int64_t id, lbm_ehd_request_info *out);
/* Fields of a finished request, as lbm_ehd_get_fields.  LBM_ESTATE if not done. */
LBM_API lbm_status lbm_ehd_server_fields(lbm_ehd_server *s, int64_t id, uint32_t mask,
                                         double *out, size_t n_doubles);
/* Forget a finished or failed request and free its device memory.
 * LBM_ESTATE while it is queued or running. */
LBM_API lbm_status lbm_ehd_server_release(lbm_ehd_server *s, int64_t id);
/* Device bytes held by admitted, unreleased requests. */
LBM_API size_t lbm_ehd_server_used_bytes(const lbm_ehd_server *s);
/* Message of the last server error on the calling thread. */
LBM_API const char *lbm_ehd_server_last_error(void);
/* Wait for the server's work and free everything it holds.  NULL allowed. */
LBM_API lbm_status lbm_ehd_server_destroy(lbm_ehd_server *s);

/* Wait for all work of the handle.  LBM_EDEVICE if a kernel failed. */
LBM_API lbm_status lbm_ehd_synchronize(lbm_ehd *h);

/* Release the handle and what the library allocated.  NULL is allowed. */
LBM_API lbm_status lbm_ehd_destroy(lbm_ehd *h);

/* Message of the last error on the calling thread ("" if none). */
LBM_API const char *lbm_ehd_last_error(void);

/* Algorithmic HBM bytes one lattice update moves in the fused sweep, each
 * item read and written once: the 32 moving populations in the storage type
 * (with 16-bit storage: 30, the rest populations of the two ions being kept
 * in FP64, plus the lines of the reference phase of h and the reference
 * potential of g), the rest populations (h0: FP64, 4 bytes with FP32
 * storage; with 16-bit storage also p0 and n0, FP64) and (phi u)(t-1) in the
 * arithmetic type.  FP64 560, FP32 280, FP32 storage with FP64 arithmetic
 * 296, FP16 192, BF16 200. */
LBM_API double lbm_ehd_bytes_per_lup(int32_t precision);

/* Measurement helper, not part of the method: copy `bytes` (a multiple of
 * 16) from device buffer src to dst on `stream` with the same raw buffer
 * instructions the sweep uses, `width` = 4 (one dword per lane) or 16 bytes
 * per lane.  Its bandwidth is the attainable HBM rate and its hardware
 * counters calibrate the sweep's.  LBM_EINVAL on a bad size or width. */
LBM_API lbm_status lbm_ehd_stream_copy(const void *src, void *dst, size_t bytes, void *stream,
                                       int32_t width);

#ifdef __cplusplus
}
#endif

#endif /* LBM_EHD_H */
