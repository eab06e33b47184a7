/*
 * lbm_ehd_oracle.c -- plain FP64 CPU oracle for the phase-field MRT lattice
 * Boltzmann method for two-phase electrohydrodynamic (EHD) flow driven by the
 * Onsager-Wien effect (Zheng, Wang, Xiong, Huang, Luo, arXiv 2501.04920).
 *
 * THIS FILE IS TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark load it.  It shares no code, header,
 * table or helper with the GPU library and must never be linked into it.
 *
 * What it computes, per time step t -> t+1 (Sec. 4 of the paper), written as
 * plainly as possible: per-cell loops, the MRT collision as the dense matrix
 * products M^-1 S M and M^-1 (I - S/2) M built from the matrices typed in from
 * Eq. (28) (D2Q9) and Eq. (46) (D2Q5), and every equilibrium and forcing term
 * written in the form the paper prints it.
 *
 *   1. optional extra Poisson (g-only) sweeps, Eq. (44)-(49)
 *   2. local moments: phi (Eq. 33), sum p, sum n (Eq. 41/43), psi (Eq. 49)
 *   3. phase-interpolated properties, Eq. (61); relaxation times Eq. (30),
 *      (37), (47), (55); delta and gamma of Eq. (5)-(6)
 *   4. isotropic finite differences for grad(phi), lap(phi), grad(psi),
 *      Eq. (59) and the Laplacian that follows it; E = -grad(psi), Eq. (9),
 *      or (option) the local field of Eq. (50) from the node's g
 *   5. ion concentrations by the explicit solve of Eq. (41)-(43) (the root
 *      of Eq. 42 in a cancellation-free form), reaction R of Eq. (5)-(6),
 *      charge density Eq. (8)
 *   6. forces: chemical potential Eq. (13), surface tension Eq. (12), electric
 *      force Eq. (14)
 *   7. velocity and pressure, Eq. (56)-(57); d(phi u)/dt by Eq. (58)
 *   8. MRT collisions of f (Eq. 51-55), h (Eq. 27-32), p and n (Eq. 34-40,
 *      on D2Q5), g (Eq. 44-47)
 *   9. streaming, periodic in x (or between side walls), with halfway wall
 *      rules at the electrodes (Eq. 64 and the boundary conditions of the 1-D
 *      test in Sec. 5.1)
 *
 * Readings taken where the paper is silent, garbled or inconsistent:
 *   - ions use the D2Q5 lattice (weights of Eq. 26, matrix N of Eq. 46) by
 *     default; with ion_q9 = 1 they use D2Q9 as Eq. (34)-(38) write them
 *     (weights of Eq. 25, matrix M of Eq. 28, s_1 = s_2 = 1/tau of Eq. 37);
 *   - which MRT rows relax with 1/tau is a per-equation bit mask; default:
 *     rows 1,2 (first moments) for h, p, n, g and rows 3,4,5 (second moments)
 *     for f, every other row relaxes with s_free (1.0 in Sec. 6);
 *   - G_i of Eq. (40) reads w_i c_i . (mu_+ c_+ / c_s^2) grad(psi), the mirror
 *     of the anion term, giving cation drift +mu_+ E and anion drift -mu_- E;
 *   - F(E) uses the field magnitude |E|;
 *   - Poisson source: (rho_e + grad(eps).grad(psi))/eps by default, whose
 *     fixed point is div(eps grad psi) = -rho_e (Eq. 7); the literal rho_e/eps
 *     of Eq. (44) is selectable;
 *   - Poisson source weights: with the weights printed in Eq. (44) the part of
 *     the source that feeds psi (Eq. 49) is (1 - w_0) theta S, and the steady
 *     state solves lap(psi) = -(1 - w_0) S instead of Eq. (7); by default the
 *     source is divided by (1 - w_0) so that the steady state solves Eq. (7),
 *     the printed weights remain selectable;
 *   - walls are halfway between lattice rows: anode (psi = dpsi) below row 0,
 *     cathode (psi = 0) above row ny-1.  f and h bounce back; g anti-bounces
 *     back with the wall potential; an ion with a zero-concentration condition
 *     anti-bounces back with 0, an ion with a zero-gradient condition
 *     anti-bounces back with the concentration of the wall node itself;
 *   - stencil ghosts: phi mirrored across the wall, psi odd about the wall
 *     value; grad(rho) and grad(eps) follow from grad(phi) by Eq. (61);
 *   - optional side walls (the other boundaries of Eq. 64: u = 0, zero normal
 *     derivative of c+, c- and psi), halfway between lattice columns at
 *     x = -1/2 and x = nx - 1/2: f bounces back (u = 0); h reflects
 *     specularly (the mirror image of the domain, a neutral wall with zero
 *     phi flux, consistent with the mirrored stencil ghosts); the ion and
 *     potential populations bounce back, which for D2Q5 is the same as
 *     specular reflection (zero flux); the stencil ghosts mirror phi and psi.
 *     Where the mirror image of an h population's source lies beyond an
 *     electrode (a corner), h bounces back;
 *   - the unit normal grad(phi)/|grad(phi)| of Eq. (1) and (32) is undefined
 *     where grad(phi) = 0, which happens where lambda of Eq. (2) is not
 *     small (the centre of a droplet, phi < 1 there); next to such a point
 *     its direction follows the rounding of grad(phi), and the step turns
 *     a 1e-15 change of one population into a 1e-5 change of phi within
 *     1000 steps.  It is evaluated as grad(phi)/sqrt(|grad(phi)|^2 + n_eps^2)
 *     (default n_eps = 1e-4 in lattice units, far below the interface's
 *     |grad(phi)| ~ 1/W); n_eps = 0 selects the bare form, taken as 0 where
 *     |grad(phi)| < 1e-12;
 *   - d(phi u)/dt at the first step uses (phi u)(t-1) = 0;
 *   - with the local field of Eq. (50), grad(psi) = -E wherever it enters
 *     (forces, reaction, ion drift, Poisson source, g-only sweeps), and
 *     tau_g is taken as printed whatever rate the g masks give the first
 *     moments.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_API __attribute__((visibility("default")))

/* ------------------------------------------------------------------------ */
/* Lattices, Eq. (25) and Eq. (26).                                          */
/* ------------------------------------------------------------------------ */
static const int CX9[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY9[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W9[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int CX5[5] = {0, 1, 0, -1, 0};
static const int CY5[5] = {0, 0, 1, 0, -1};
static const double W5[5] = {1.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0};
static const double CS2 = 1.0 / 3.0; /* c_s^2 with c = dx/dt = 1 */

/* Transformation matrix of Eq. (28), typed in row by row. */
static const double M9[81] = {
    1, 1, 1, 1, 1, 1, 1, 1, 1,
    0, 1, 0, -1, 0, 1, -1, -1, 1,
    0, 0, 1, 0, -1, 1, 1, -1, -1,
    0, 1, 0, 1, 0, 1, 1, 1, 1,
    0, 0, 1, 0, 1, 1, 1, 1, 1,
    0, 0, 0, 0, 0, 1, -1, 1, -1,
    0, 0, 0, 0, 0, 1, -1, -1, 1,
    0, 0, 0, 0, 0, 1, 1, -1, -1,
    0, 0, 0, 0, 0, 1, 1, 1, 1};

/* Transformation matrix of Eq. (46), typed in row by row. */
static const double N5[25] = {
    1, 1, 1, 1, 1,
    0, 1, 0, -1, 0,
    0, 0, 1, 0, -1,
    0, 1, 0, 1, 0,
    0, 0, 1, 0, 1};

/* Population sets, stored one after the other: f (9), h (9), p, n (5 each,
 * or 9 each with D2Q9 ions), g (5).  The offsets of p, n and g and the
 * number of populations are in the state (op, on, og, npop). */
enum { OF_F = 0, OF_H = 9, OF_P = 18 };

enum { WALLS_ELECTRODES = 0, WALLS_INSULATING = 1, WALLS_PERIODIC = 2 };

/* Field indices of orc_fields(). */
enum {
  FLD_PHI = 0, FLD_PSI, FLD_CP, FLD_CM, FLD_RHOE, FLD_UX, FLD_UY, FLD_P,
  FLD_EX, FLD_EY, NFIELD
};

typedef struct {
  int32_t nx, ny;
  int32_t walls;         /* 0 electrodes, 1 electrodes with ion-tight walls, 2 periodic y */
  int32_t reaction;      /* 1: R of Eq. (5); 0: R = 0 (leaky-dielectric limit, Sec. 5.2) */
  int32_t poisson_form;  /* 1: source (rho_e + grad eps . grad psi)/eps; 0: rho_e/eps */
  int32_t flow;          /* 1: solve Eq. (51); 0: u = 0, f left untouched */
  int32_t ion_force;     /* 1: keep L_i of Eq. (39); 0: drop it */
  int32_t poisson_iters; /* extra g-only sweeps before every step */
  int32_t mask_f, mask_h, mask_p, mask_n, mask_g; /* MRT rows relaxed with 1/tau */
  int32_t poisson_norm;  /* 1: source weights w_i/(1 - w_0); 0: w_i as printed in Eq. (44) */
  int32_t side_walls;    /* 0: periodic in x; 1: side walls of Eq. (64) at x = -1/2, nx - 1/2 */
  int32_t local_field;   /* 0: E = -grad psi by Eq. (59); 1: E from the g populations, Eq. (50) */
  double rho_v, rho_r;   /* density of the outer (v) phase and ratio l/v, Eq. (60) */
  double eta_v, eta_r;   /* dynamic viscosity and ratio */
  double M_phi, W, zeta; /* Allen-Cahn mobility, interface width, surface tension */
  double theta;          /* artificial diffusion of the Poisson LBE, Eq. (47) */
  double dpsi;           /* anode potential; the cathode is at 0 */
  double eps_v, eps_r;   /* permittivity and ratio */
  double mu_v, mu_r;     /* cation mobility (outer phase) and ratio l/v */
  double m_ratio;        /* mu_- / mu_+ */
  double v_th;           /* k_B T / e_0: D = v_th * mu (Einstein relation, Sec. 2.2) */
  double c0;             /* zero-field concentration */
  double q;              /* elementary charge e_0 in lattice units */
  double gamma_v;        /* Onsager constant of Eq. (6) in the outer phase */
  double force_x, force_y; /* external body-force density (tests) */
  double s_free;         /* rate of the free MRT rows */
  double n_eps;          /* regularisation of the unit normal (0: bare form) */
  int32_t ion_q9;        /* 0: ions on D2Q5; 1: ions on D2Q9, Eq. (34)-(38) as printed */
  int32_t reserved;
} orc_params;

typedef struct {
  orc_params P;
  int nx, ny;
  size_t nc;
  double *pop;   /* [33][ny][nx] populations at the current time, before collision */
  double *post;  /* [33][ny][nx] post-collision populations */
  double *jprev; /* [2][ny][nx] phi*u of the previous step, for Eq. (58) */
  double *phi, *psi, *sp, *sn; /* moment fields */
  double *cp, *cm; /* concentrations at the collision time, for the wall rules */
  long step;
  double M9i[81], N5i[25];
  int opp9[9], opp5[5];
  int mirx9[9];  /* direction with c_x reversed */
  int qi;        /* ion lattice: 5 or 9 populations per species */
  int op, on, og, npop; /* offsets of p, n, g; populations per cell */
} orc_state;

/* Macroscopic quantities at one node, steps 3-7. */
typedef struct {
  double phi, P, Q, psi;
  double rho, eta, eps, mup, mum;
  double tau_f, tau_h, tau_p, tau_n, tau_g;
  double delta, gamma;
  double gphi[2], lphi, gpsi[2], E[2];
  double Fo, cbp, cbm, cp, cm, R, rhoe;
  double mu_phi, grho[2], geps[2], F[2];
  double u[2], p;
} macro_t;

/* ------------------------------------------------------------------------ */
/* Small dense linear algebra.                                               */
/* ------------------------------------------------------------------------ */
static int invert(int n, const double *A, double *Ainv) {
  double a[81 * 2];
  int w = 2 * n;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < w; ++j)
      a[i * w + j] = j < n ? A[i * n + j] : (j - n == i ? 1.0 : 0.0);
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (fabs(a[r * w + c]) > fabs(a[piv * w + c])) piv = r;
    if (a[piv * w + c] == 0.0) return -1;
    if (piv != c)
      for (int j = 0; j < w; ++j) {
        double t = a[c * w + j];
        a[c * w + j] = a[piv * w + j];
        a[piv * w + j] = t;
      }
    double d = a[c * w + c];
    for (int j = 0; j < w; ++j) a[c * w + j] /= d;
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = a[r * w + c];
      if (f != 0.0)
        for (int j = 0; j < w; ++j) a[r * w + j] -= f * a[c * w + j];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Ainv[i * n + j] = a[i * w + n + j];
  return 0;
}

/* A = Minv diag(s) M and B = Minv (I - diag(s)/2) M. */
static void mrt_operators(int q, const double *M, const double *Minv, const double *s,
                          double *A, double *B) {
  for (int i = 0; i < q; ++i)
    for (int j = 0; j < q; ++j) {
      double a = 0.0, b = 0.0;
      for (int k = 0; k < q; ++k) {
        a += Minv[i * q + k] * s[k] * M[k * q + j];
        b += Minv[i * q + k] * (1.0 - 0.5 * s[k]) * M[k * q + j];
      }
      A[i * q + j] = a;
      B[i * q + j] = b;
    }
}

/* The operators only depend on the rate vector; keep the last one built for
 * each population set so that a row of cells with the same rates does not
 * rebuild them.  The cached matrices are the ones mrt_operators() returns. */
typedef struct {
  int valid[5];
  double s[5][9];
  double A[5][81], B[5][81];
} mrt_memo;

static void mrt_cached(mrt_memo *mm, int slot, int q, const double *M, const double *Minv,
                       const double *s, const double **A, const double **B) {
  int same = mm->valid[slot];
  for (int k = 0; same && k < q; ++k) same = mm->s[slot][k] == s[k];
  if (!same) {
    mrt_operators(q, M, Minv, s, mm->A[slot], mm->B[slot]);
    memcpy(mm->s[slot], s, q * sizeof(double));
    mm->valid[slot] = 1;
  }
  *A = mm->A[slot];
  *B = mm->B[slot];
}

static void matvec(int q, const double *A, const double *x, double *y) {
  for (int i = 0; i < q; ++i) {
    double acc = 0.0;
    for (int j = 0; j < q; ++j) acc += A[i * q + j] * x[j];
    y[i] = acc;
  }
}

/* Relaxation rates: rows in `mask` take 1/tau, the rest s_free. */
static void rates(int q, int mask, double tau, double s_free, double *s) {
  for (int k = 0; k < q; ++k) s[k] = ((mask >> k) & 1) ? 1.0 / tau : s_free;
}

/* ------------------------------------------------------------------------ */
/* Equilibria and forcing terms, one function per printed equation.          */
/* ------------------------------------------------------------------------ */

/* Eq. (53). */
static double r_i(int i, const double *u) {
  double cu = CX9[i] * u[0] + CY9[i] * u[1];
  double uu = u[0] * u[0] + u[1] * u[1];
  return W9[i] * (cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
}

/* Eq. (52). */
static void feq(double p, double rho, const double *u, double *out) {
  for (int i = 0; i < 9; ++i)
    out[i] = (i == 0 ? (W9[0] - 1.0) : W9[i]) * p / CS2 + rho * r_i(i, u);
}

/* Eq. (54). */
static void fforce(const double *u, const double *grho, const double *F, double *out) {
  double ugr = u[0] * grho[0] + u[1] * grho[1];
  for (int i = 0; i < 9; ++i) {
    double c[2] = {CX9[i], CY9[i]};
    double cF = c[0] * F[0] + c[1] * F[1];
    /* (u grad rho) : (c c - c_s^2 I) */
    double dd = 0.0;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        dd += u[a] * grho[b] * (c[a] * c[b] - (a == b ? CS2 : 0.0));
    out[i] = W9[i] * (ugr + cF / CS2 + dd / CS2);
  }
}

/* Eq. (31). */
static void heq(double phi, const double *u, double *out) {
  for (int i = 0; i < 9; ++i)
    out[i] = W9[i] * phi * (1.0 + (CX9[i] * u[0] + CY9[i] * u[1]) / CS2);
}

/* Eq. (32): dJ = d(phi u)/dt, nhat = grad(phi)/|grad(phi)|. */
/* The unit normal grad(phi)/|grad(phi)| of Eq. (1) and (32), regularised
 * as grad(phi)/sqrt(|grad(phi)|^2 + n_eps^2); n_eps = 0: the bare form,
 * taken as 0 where |grad(phi)| < 1e-12. */
static void unit_normal(const double g[2], double n_eps, double n[2]) {
  double g2 = g[0] * g[0] + g[1] * g[1];
  if (n_eps > 0.0) {
    double d = sqrt(g2 + n_eps * n_eps);
    n[0] = g[0] / d;
    n[1] = g[1] / d;
  } else if (sqrt(g2) >= 1e-12) {
    double d = sqrt(g2);
    n[0] = g[0] / d;
    n[1] = g[1] / d;
  } else {
    n[0] = n[1] = 0.0;
  }
}

static void hforce(const double *dJ, const double *nhat, double phi, double W, double *out) {
  double lam = 4.0 * phi * (1.0 - phi) / W; /* Eq. (2) */
  for (int i = 0; i < 9; ++i) {
    double vx = dJ[0] + CS2 * nhat[0] * lam;
    double vy = dJ[1] + CS2 * nhat[1] * lam;
    out[i] = W9[i] * (CX9[i] * vx + CY9[i] * vy) / CS2;
  }
}

/* The lattice of q velocities (5: D2Q5 of Eq. 26, 9: D2Q9 of Eq. 25). */
static const int *lat_cx(int q) { return q == 9 ? CX9 : CX5; }
static const int *lat_cy(int q) { return q == 9 ? CY9 : CY5; }
static const double *lat_w(int q) { return q == 9 ? W9 : W5; }

/* Eq. (38) on the ion lattice of q velocities. */
static void ioneq(int q, double c, const double *u, double *out) {
  const int *cx = lat_cx(q), *cy = lat_cy(q);
  const double *w = lat_w(q);
  for (int i = 0; i < q; ++i)
    out[i] = w[i] * c * (1.0 + (cx[i] * u[0] + cy[i] * u[1]) / CS2);
}

/* Eq. (39): R_i + L_i for one species with concentration c. */
static void ionsrc(int q, double R, double c, const double *F, int with_L, double *out) {
  const int *cx = lat_cx(q), *cy = lat_cy(q);
  const double *w = lat_w(q);
  for (int i = 0; i < q; ++i) {
    double L = with_L ? w[i] * (cx[i] * c * F[0] + cy[i] * c * F[1]) / CS2 : 0.0;
    out[i] = w[i] * R + L;
  }
}

/* Eq. (40): G_i (mobility mu, concentration c). */
static void iondrift(int q, double mu, double c, const double *gpsi, double *out) {
  const int *cx = lat_cx(q), *cy = lat_cy(q);
  const double *w = lat_w(q);
  for (int i = 0; i < q; ++i)
    out[i] = w[i] * (cx[i] * gpsi[0] + cy[i] * gpsi[1]) * mu * c / CS2;
}

/* Eq. (45). */
static void geq(double psi, double *out) {
  for (int i = 0; i < 5; ++i) out[i] = (i == 0 ? (W5[0] - 1.0) : W5[i]) * psi;
}

/* Eq. (42) with Eq. (43): c+ is the non-negative root of
 * lam0 c+^2 + b c+ - cb+ = 0 with b = 1 - lam0 (cb+ - cb-).  Eq. (42) writes it
 * as (-b + sqrt(b^2 + 4 lam0 cb+)) / (2 lam0), which cancels when b > 0 and
 * lam0 is small; there the equal form 2 cb+ / (b + sqrt(...)) is used (it is
 * also finite at lam0 = 0).  Then c- = c+ - cb+ + cb-. */
static void ion_solve(double cbp, double cbm, double lam0, double *cp, double *cm) {
  double b = 1.0 - lam0 * (cbp - cbm);
  double root = sqrt(b * b + 4.0 * lam0 * cbp);
  if (b >= 0.0)
    *cp = 2.0 * cbp / (b + root);
  else
    *cp = (root - b) / (2.0 * lam0);
  *cm = *cp - cbp + cbm;
}

/* ------------------------------------------------------------------------ */
/* Helpers on the grid.                                                      */
/* ------------------------------------------------------------------------ */
static inline size_t cidx(const orc_state *s, int x, int y) { return (size_t)y * s->nx + x; }
static inline int wrapx(const orc_state *s, int x) { return (x % s->nx + s->nx) % s->nx; }

enum { GHOST_MIRROR = 0, GHOST_ODD = 1 };

/* Field value at (x, y), x or y possibly one step outside the domain. */
static double field_at(const orc_state *s, const double *f, int ghost, int x, int y) {
  if (s->P.side_walls)
    x = x < 0 ? 0 : (x >= s->nx ? s->nx - 1 : x); /* mirrored across a side wall */
  else
    x = wrapx(s, x);
  if (y >= 0 && y < s->ny) return f[cidx(s, x, y)];
  if (s->P.walls == WALLS_PERIODIC) return f[cidx(s, x, (y % s->ny + s->ny) % s->ny)];
  int yin = y < 0 ? 0 : s->ny - 1;
  double v = f[cidx(s, x, yin)];
  if (ghost == GHOST_MIRROR) return v;
  double psi_w = y < 0 ? s->P.dpsi : 0.0;
  return 2.0 * psi_w - v;
}

/* Eq. (59) and the isotropic Laplacian below it, dt = 1. */
static void stencil(const orc_state *s, const double *f, int ghost, int x, int y, double *grad,
                    double *lap) {
  double c0 = f[cidx(s, x, y)];
  double gx = 0.0, gy = 0.0, l = 0.0;
  for (int i = 1; i < 9; ++i) {
    double v = field_at(s, f, ghost, x + CX9[i], y + CY9[i]);
    gx += W9[i] * CX9[i] * v / CS2;
    gy += W9[i] * CY9[i] * v / CS2;
    l += 2.0 * W9[i] * (v - c0) / CS2;
  }
  grad[0] = gx;
  grad[1] = gy;
  if (lap) *lap = l;
}

static void compute_moments(orc_state *s) {
  for (size_t c = 0; c < s->nc; ++c) {
    double phi = 0.0, P = 0.0, Q = 0.0, gs = 0.0;
    for (int i = 0; i < 9; ++i) phi += s->pop[(OF_H + i) * s->nc + c];   /* Eq. (33) */
    for (int i = 0; i < s->qi; ++i) P += s->pop[(s->op + i) * s->nc + c];
    for (int i = 0; i < s->qi; ++i) Q += s->pop[(s->on + i) * s->nc + c];
    for (int i = 1; i < 5; ++i) gs += s->pop[(s->og + i) * s->nc + c];
    s->phi[c] = phi;
    s->sp[c] = P;
    s->sn[c] = Q;
    s->psi[c] = gs / (1.0 - W5[0]); /* Eq. (49) */
  }
}

/* Eq. (50): the field from the first moment of the node's incoming g,
 * E = sum_i c_i g_i / (c_s^2 tau_g). */
static void field_from_g(const orc_state *s, size_t c, double tau_g, double *E) {
  double ex = 0.0, ey = 0.0;
  for (int i = 1; i < 5; ++i) {
    double g = s->pop[(s->og + i) * s->nc + c];
    ex += CX5[i] * g;
    ey += CY5[i] * g;
  }
  E[0] = ex / (CS2 * tau_g);
  E[1] = ey / (CS2 * tau_g);
}

/* Steps 3-7 at one node.  Needs the moment fields of the current time. */
static void macro_at(const orc_state *s, int x, int y, macro_t *m) {
  const orc_params *P = &s->P;
  size_t c = cidx(s, x, y);
  m->phi = s->phi[c];
  m->P = s->sp[c];
  m->Q = s->sn[c];
  m->psi = s->psi[c];

  /* Eq. (60)-(61): linear interpolation of every phase property. */
  double rho_l = P->rho_v * P->rho_r, eta_l = P->eta_v * P->eta_r;
  double eps_l = P->eps_v * P->eps_r, mu_l = P->mu_v * P->mu_r;
  m->rho = m->phi * (rho_l - P->rho_v) + P->rho_v;
  m->eta = m->phi * (eta_l - P->eta_v) + P->eta_v;
  m->eps = m->phi * (eps_l - P->eps_v) + P->eps_v;
  m->mup = m->phi * (mu_l - P->mu_v) + P->mu_v;
  m->mum = P->m_ratio * m->mup;

  /* Relaxation times, Eq. (30), (37), (47), (55). */
  double Dp = P->v_th * m->mup, Dm = P->v_th * m->mum;
  m->tau_f = 0.5 + m->eta / (m->rho * CS2);
  m->tau_h = 0.5 + P->M_phi / CS2;
  m->tau_p = 0.5 + Dp / CS2;
  m->tau_n = 0.5 + Dm / CS2;
  m->tau_g = 0.5 + P->theta / CS2;

  /* delta = e0 (mu+ + mu-)/eps (Eq. 5); gamma proportional to 1/eps (Eq. 6). */
  m->delta = P->q * (m->mup + m->mum) / m->eps;
  m->gamma = P->gamma_v * P->eps_v / m->eps;

  /* Finite differences, Eq. (59); E = -grad psi, Eq. (9), or with the local
   * field E from Eq. (50) and grad psi = -E wherever it appears. */
  stencil(s, s->phi, GHOST_MIRROR, x, y, m->gphi, &m->lphi);
  if (P->local_field) {
    field_from_g(s, c, m->tau_g, m->E);
    m->gpsi[0] = -m->E[0];
    m->gpsi[1] = -m->E[1];
  } else {
    stencil(s, s->psi, GHOST_ODD, x, y, m->gpsi, NULL);
    m->E[0] = -m->gpsi[0];
    m->E[1] = -m->gpsi[1];
  }

  /* Ions, Eq. (5), (6), (8), (41)-(43). */
  double Emag = sqrt(m->E[0] * m->E[0] + m->E[1] * m->E[1]);
  m->Fo = 1.0 + 2.0 * m->gamma * Emag;
  if (P->reaction) {
    double lam0 = 0.5 * m->delta;
    m->cbp = m->P + 0.5 * m->delta * P->c0 * P->c0 * m->Fo;
    m->cbm = m->Q + 0.5 * m->delta * P->c0 * P->c0 * m->Fo;
    ion_solve(m->cbp, m->cbm, lam0, &m->cp, &m->cm);
    m->R = m->delta * (P->c0 * P->c0 * m->Fo - m->cp * m->cm);
  } else {
    m->cbp = m->P;
    m->cbm = m->Q;
    m->cp = m->P;
    m->cm = m->Q;
    m->R = 0.0;
  }
  m->rhoe = P->q * (m->cp - m->cm);

  /* Forces, Eq. (12)-(14). */
  double beta_ac = 12.0 * P->zeta / P->W, kappa = 1.5 * P->zeta * P->W;
  m->mu_phi = 4.0 * beta_ac * m->phi * (m->phi - 1.0) * (m->phi - 0.5) - kappa * m->lphi;
  for (int a = 0; a < 2; ++a) {
    m->grho[a] = (rho_l - P->rho_v) * m->gphi[a];
    m->geps[a] = (eps_l - P->eps_v) * m->gphi[a];
  }
  double E2 = m->E[0] * m->E[0] + m->E[1] * m->E[1];
  double Fext[2] = {P->force_x, P->force_y};
  for (int a = 0; a < 2; ++a)
    m->F[a] = m->mu_phi * m->gphi[a] - 0.5 * E2 * m->geps[a] + m->rhoe * m->E[a] + Fext[a];

  /* Velocity and pressure, Eq. (56)-(57). */
  if (P->flow) {
    double jx = 0.0, jy = 0.0, sum_nz = 0.0;
    for (int i = 0; i < 9; ++i) {
      double fi = s->pop[(OF_F + i) * s->nc + c];
      jx += CX9[i] * fi;
      jy += CY9[i] * fi;
      if (i != 0) sum_nz += fi;
    }
    m->u[0] = (jx + 0.5 * m->F[0]) / m->rho;
    m->u[1] = (jy + 0.5 * m->F[1]) / m->rho;
    double ugr = m->u[0] * m->grho[0] + m->u[1] * m->grho[1];
    m->p = CS2 / (1.0 - W9[0]) * (sum_nz + 0.5 * ugr + m->rho * r_i(0, m->u));
  } else {
    m->u[0] = m->u[1] = 0.0;
    m->p = 0.0;
  }
}

/* Steps 3-8 at one node: writes post-collision populations. */
static void collide_at(orc_state *s, int x, int y, mrt_memo *mm) {
  const orc_params *P = &s->P;
  size_t c = cidx(s, x, y), nc = s->nc;
  macro_t m;
  macro_at(s, x, y, &m);
  s->cp[c] = m.cp;
  s->cm[c] = m.cm;

  /* Eq. (58). */
  double J[2] = {m.phi * m.u[0], m.phi * m.u[1]};
  double dJ[2] = {J[0] - s->jprev[c], J[1] - s->jprev[nc + c]};
  s->jprev[c] = J[0];
  s->jprev[nc + c] = J[1];

  const double *A9, *B9, *A5, *B5;
  double sv[9];
  double x9[9], e9[9], d9[9], s9[9], t9[9], t9b[9];
  double x5[5], e5[5], d5[5], t5[5];

  /* f, Eq. (51). */
  for (int i = 0; i < 9; ++i) x9[i] = s->pop[(OF_F + i) * nc + c];
  if (P->flow) {
    rates(9, P->mask_f, m.tau_f, P->s_free, sv);
    mrt_cached(mm, 0, 9, M9, s->M9i, sv, &A9, &B9);
    feq(m.p, m.rho, m.u, e9);
    fforce(m.u, m.grho, m.F, s9);
    for (int i = 0; i < 9; ++i) d9[i] = x9[i] - e9[i];
    matvec(9, A9, d9, t9);
    matvec(9, B9, s9, t9b);
    for (int i = 0; i < 9; ++i) s->post[(OF_F + i) * nc + c] = x9[i] - t9[i] + t9b[i];
  } else {
    for (int i = 0; i < 9; ++i) s->post[(OF_F + i) * nc + c] = x9[i];
  }

  /* h, Eq. (27) with Eq. (29)-(32). */
  double nhat[2];
  unit_normal(m.gphi, P->n_eps, nhat);
  for (int i = 0; i < 9; ++i) x9[i] = s->pop[(OF_H + i) * nc + c];
  rates(9, P->mask_h, m.tau_h, P->s_free, sv);
  mrt_cached(mm, 1, 9, M9, s->M9i, sv, &A9, &B9);
  heq(m.phi, m.u, e9);
  hforce(dJ, nhat, m.phi, P->W, s9);
  for (int i = 0; i < 9; ++i) d9[i] = x9[i] - e9[i];
  matvec(9, A9, d9, t9);
  matvec(9, B9, s9, t9b);
  for (int i = 0; i < 9; ++i) s->post[(OF_H + i) * nc + c] = x9[i] - t9[i] + t9b[i];

  /* Ions on the lattice of qi velocities, with its transformation matrix
   * (M of Eq. 28 for D2Q9, N of Eq. 46 for D2Q5). */
  const int qi = s->qi;
  const double *MI = qi == 9 ? M9 : N5, *MIi = qi == 9 ? s->M9i : s->N5i;
  const double *AI, *BI;
  double xi[9], ei[9], di[9], si[9], gi[9], ti[9], tib[9], tig[9];

  /* p (cations), Eq. (34): - M^-1 S M G. */
  for (int i = 0; i < qi; ++i) xi[i] = s->pop[(s->op + i) * nc + c];
  rates(qi, P->mask_p, m.tau_p, P->s_free, sv);
  mrt_cached(mm, 2, qi, MI, MIi, sv, &AI, &BI);
  ioneq(qi, m.cp, m.u, ei);
  ionsrc(qi, m.R, m.cp, m.F, P->ion_force, si);
  iondrift(qi, m.mup, m.cp, m.gpsi, gi);
  for (int i = 0; i < qi; ++i) di[i] = xi[i] - ei[i];
  matvec(qi, AI, di, ti);
  matvec(qi, BI, si, tib);
  matvec(qi, AI, gi, tig);
  for (int i = 0; i < qi; ++i) s->post[(s->op + i) * nc + c] = xi[i] - ti[i] + tib[i] - tig[i];

  /* n (anions), Eq. (35): + M^-1 S M Gbar. */
  for (int i = 0; i < qi; ++i) xi[i] = s->pop[(s->on + i) * nc + c];
  rates(qi, P->mask_n, m.tau_n, P->s_free, sv);
  mrt_cached(mm, 3, qi, MI, MIi, sv, &AI, &BI);
  ioneq(qi, m.cm, m.u, ei);
  ionsrc(qi, m.R, m.cm, m.F, P->ion_force, si);
  iondrift(qi, m.mum, m.cm, m.gpsi, gi);
  for (int i = 0; i < qi; ++i) di[i] = xi[i] - ei[i];
  matvec(qi, AI, di, ti);
  matvec(qi, BI, si, tib);
  matvec(qi, AI, gi, tig);
  for (int i = 0; i < qi; ++i) s->post[(s->on + i) * nc + c] = xi[i] - ti[i] + tib[i] + tig[i];

  /* g, Eq. (44)-(47). */
  double Spsi = P->poisson_form
                    ? (m.rhoe + m.geps[0] * m.gpsi[0] + m.geps[1] * m.gpsi[1]) / m.eps
                    : m.rhoe / m.eps;
  for (int i = 0; i < 5; ++i) x5[i] = s->pop[(s->og + i) * nc + c];
  rates(5, P->mask_g, m.tau_g, P->s_free, sv);
  mrt_cached(mm, 4, 5, N5, s->N5i, sv, &A5, &B5);
  geq(m.psi, e5);
  for (int i = 0; i < 5; ++i) d5[i] = x5[i] - e5[i];
  matvec(5, A5, d5, t5);
  double wn = P->poisson_norm ? 1.0 / (1.0 - W5[0]) : 1.0;
  for (int i = 0; i < 5; ++i)
    s->post[(s->og + i) * nc + c] = x5[i] - t5[i] + wn * W5[i] * Spsi * P->theta;
}

/* One g-only sweep with phi and rho_e = e0 (sum p - sum n) held fixed. */
static void poisson_collide_at(orc_state *s, int x, int y, mrt_memo *mm) {
  const orc_params *P = &s->P;
  size_t c = cidx(s, x, y), nc = s->nc;
  double eps_l = P->eps_v * P->eps_r;
  double phi = s->phi[c];
  double eps = phi * (eps_l - P->eps_v) + P->eps_v;
  double tau_g = 0.5 + P->theta / CS2;
  double rhoe = P->q * (s->sp[c] - s->sn[c]);
  double gphi[2], gpsi[2];
  stencil(s, s->phi, GHOST_MIRROR, x, y, gphi, NULL);
  if (P->local_field) {
    double E[2];
    field_from_g(s, c, tau_g, E);
    gpsi[0] = -E[0];
    gpsi[1] = -E[1];
  } else {
    stencil(s, s->psi, GHOST_ODD, x, y, gpsi, NULL);
  }
  double geps[2] = {(eps_l - P->eps_v) * gphi[0], (eps_l - P->eps_v) * gphi[1]};
  double Spsi = P->poisson_form ? (rhoe + geps[0] * gpsi[0] + geps[1] * gpsi[1]) / eps
                                : rhoe / eps;
  double sv[5], x5[5], e5[5], d5[5], t5[5];
  const double *A5, *B5;
  for (int i = 0; i < 5; ++i) x5[i] = s->pop[(s->og + i) * nc + c];
  rates(5, P->mask_g, tau_g, P->s_free, sv);
  mrt_cached(mm, 4, 5, N5, s->N5i, sv, &A5, &B5);
  geq(s->psi[c], e5);
  for (int i = 0; i < 5; ++i) d5[i] = x5[i] - e5[i];
  matvec(5, A5, d5, t5);
  double wn = P->poisson_norm ? 1.0 / (1.0 - W5[0]) : 1.0;
  for (int i = 0; i < 5; ++i)
    s->post[(s->og + i) * nc + c] = x5[i] - t5[i] + wn * W5[i] * Spsi * P->theta;
}

/* Population arriving at (x, y) along direction i of a set whose source
 * node lies outside the domain: halfway wall rules. */
static double wall_rule(const orc_state *s, int set, int i, int x, int y, int bottom) {
  size_t c = cidx(s, x, y), nc = s->nc;
  int walls = s->P.walls;
  if (set == OF_F || set == OF_H)
    return s->post[(set + s->opp9[i]) * nc + c]; /* bounce-back: u = 0, no phi flux */
  if (set == s->op || set == s->on) {
    const int *opp = s->qi == 9 ? s->opp9 : s->opp5;
    const double *w = lat_w(s->qi);
    double v = s->post[(set + opp[i]) * nc + c];
    if (walls == WALLS_INSULATING) return v;
    if (set == s->op) {
      if (bottom) return -v;                     /* anode: c+ = 0 */
      return -v + 2.0 * w[i] * s->cp[c];         /* cathode: d c+/dn = 0 */
    }
    if (bottom) return -v + 2.0 * w[i] * s->cm[c]; /* anode: d c-/dn = 0 */
    return -v;                                      /* cathode: c- = 0 */
  }
  { /* g: Dirichlet potential */
    double v = s->post[(s->og + s->opp5[i]) * nc + c];
    double psi_w = bottom ? s->P.dpsi : 0.0;
    return -v + 2.0 * W5[i] * psi_w;
  }
}

static void stream_set(orc_state *s, int set, int q) {
  const int *cx = q == 9 ? CX9 : CX5, *cy = q == 9 ? CY9 : CY5;
  int nx = s->nx, ny = s->ny;
  size_t nc = s->nc;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x)
      for (int i = 0; i < q; ++i) {
        int sx = x - cx[i];
        int sy = y - cy[i];
        double v;
        if (s->P.side_walls && (sx < 0 || sx >= nx)) {
          const int *opp = q == 9 ? s->opp9 : s->opp5;
          int my = sy;   /* row of the mirror image of the source */
          if (s->P.walls == WALLS_PERIODIC) my = (my + ny) % ny;
          if (set == OF_H && my >= 0 && my < ny) {
            /* phase field: specular reflection, the population of the mirror
             * image of the source, direction mirrored in x */
            s->pop[(set + i) * nc + cidx(s, x, y)] =
                s->post[(set + s->mirx9[i]) * nc + cidx(s, x, my)];
          } else {
            /* u = 0 (and a corner for h): bounce-back of the node's own
             * opposite population; for the D2Q5 sets (no diagonals) the
             * same as specular reflection */
            s->pop[(set + i) * nc + cidx(s, x, y)] =
                s->post[(set + opp[i]) * nc + cidx(s, x, y)];
          }
          continue;
        }
        sx = wrapx(s, sx);
        if (sy >= 0 && sy < ny)
          v = s->post[(set + i) * nc + cidx(s, sx, sy)];
        else if (s->P.walls == WALLS_PERIODIC)
          v = s->post[(set + i) * nc + cidx(s, sx, (sy + ny) % ny)];
        else
          v = wall_rule(s, set, i, x, y, sy < 0);
        s->pop[(set + i) * nc + cidx(s, x, y)] = v;
      }
}

static void poisson_sweep(orc_state *s) {
  compute_moments(s);
#pragma omp parallel for schedule(static)
  for (int y = 0; y < s->ny; ++y) {
    mrt_memo mm;
    memset(mm.valid, 0, sizeof mm.valid);
    for (int x = 0; x < s->nx; ++x) poisson_collide_at(s, x, y, &mm);
  }
  stream_set(s, s->og, 5);
}

/* ------------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea, Flood 2014; reference C by S. Vigna): the n-th   */
/* output (n >= 1) of the generator started at `seed`.                       */
/* ------------------------------------------------------------------------ */
ORC_API uint64_t orc_splitmix64(uint64_t seed, uint64_t n) {
  uint64_t z = seed + n * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* Uniform in [-1, 1) from the top 53 bits. */
ORC_API double orc_noise(uint64_t seed, uint64_t n) {
  return 2.0 * ((double)(orc_splitmix64(seed, n) >> 11) * 0x1.0p-53) - 1.0;
}

/* ------------------------------------------------------------------------ */
/* Public interface.                                                         */
/* ------------------------------------------------------------------------ */
ORC_API int orc_sizeof_params(void) { return (int)sizeof(orc_params); }

ORC_API void orc_params_default(orc_params *p) {
  memset(p, 0, sizeof(*p));
  p->nx = p->ny = 128;
  p->walls = WALLS_ELECTRODES;
  p->reaction = 1;
  p->poisson_form = 1;
  p->flow = 1;
  p->ion_force = 1;
  p->poisson_iters = 0;
  p->poisson_norm = 1;
  p->mask_f = (1 << 3) | (1 << 4) | (1 << 5);
  p->mask_h = p->mask_p = p->mask_n = p->mask_g = (1 << 1) | (1 << 2);
  p->rho_v = 1.0;
  p->rho_r = 1.0;
  p->eta_v = 0.1;
  p->eta_r = 1.0;
  p->M_phi = 0.1;
  p->W = 4.0;
  p->zeta = 1e-3;
  p->theta = 0.3;
  p->dpsi = 0.0;
  p->eps_v = 1.0;
  p->eps_r = 1.0;
  p->mu_v = 0.0;
  p->mu_r = 1.0;
  p->m_ratio = 1.0;
  p->v_th = 0.0;
  p->c0 = 1.0;
  p->q = 0.0;
  p->gamma_v = 0.0;
  p->s_free = 1.0;
  p->n_eps = 1e-4;
}

ORC_API orc_state *orc_create(const orc_params *p) {
  if (p->nx < 1 || p->ny < 1) return NULL;
  orc_state *s = (orc_state *)calloc(1, sizeof(orc_state));
  if (!s) return NULL;
  s->P = *p;
  s->nx = p->nx;
  s->ny = p->ny;
  s->nc = (size_t)p->nx * p->ny;
  s->qi = p->ion_q9 ? 9 : 5;
  s->op = OF_P;
  s->on = OF_P + s->qi;
  s->og = OF_P + 2 * s->qi;
  s->npop = s->og + 5;
  s->pop = (double *)calloc((size_t)s->npop * s->nc, sizeof(double));
  s->post = (double *)calloc((size_t)s->npop * s->nc, sizeof(double));
  s->jprev = (double *)calloc(2 * s->nc, sizeof(double));
  s->phi = (double *)calloc(s->nc, sizeof(double));
  s->psi = (double *)calloc(s->nc, sizeof(double));
  s->sp = (double *)calloc(s->nc, sizeof(double));
  s->sn = (double *)calloc(s->nc, sizeof(double));
  s->cp = (double *)calloc(s->nc, sizeof(double));
  s->cm = (double *)calloc(s->nc, sizeof(double));
  if (!s->pop || !s->post || !s->jprev || !s->phi || !s->psi || !s->sp || !s->sn || !s->cp ||
      !s->cm || invert(9, M9, s->M9i) || invert(5, N5, s->N5i)) {
    free(s->pop); free(s->post); free(s->jprev); free(s->phi); free(s->psi);
    free(s->sp); free(s->sn); free(s->cp); free(s->cm); free(s);
    return NULL;
  }
  for (int i = 0; i < 9; ++i)
    for (int j = 0; j < 9; ++j) {
      if (CX9[j] == -CX9[i] && CY9[j] == -CY9[i]) s->opp9[i] = j;
      if (CX9[j] == -CX9[i] && CY9[j] == CY9[i]) s->mirx9[i] = j;
    }
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j)
      if (CX5[j] == -CX5[i] && CY5[j] == -CY5[i]) s->opp5[i] = j;
  return s;
}

ORC_API void orc_destroy(orc_state *s) {
  if (!s) return;
  free(s->pop); free(s->post); free(s->jprev); free(s->phi); free(s->psi);
  free(s->sp); free(s->sn); free(s->cp); free(s->cm);
  free(s);
}

/* Initial state: a centred tanh droplet (the exact 1-D equilibrium of
 * Eq. (1)-(2)), fluid at rest with zero pressure, equilibrium ion
 * populations at c0 (1 + noise xi), xi from SplitMix64 output 2k+1 (cations)
 * and 2k+2 (anions) of cell k = y nx + x, and the potential linear between the
 * electrodes (zero in a y-periodic box). */
ORC_API void orc_init_droplet(orc_state *s, double xc, double yc, double R, double noise,
                              uint64_t seed) {
  const orc_params *P = &s->P;
  size_t nc = s->nc;
  double zero_u[2] = {0.0, 0.0};
  for (int y = 0; y < s->ny; ++y)
    for (int x = 0; x < s->nx; ++x) {
      size_t c = cidx(s, x, y);
      double r = sqrt((x - xc) * (x - xc) + (y - yc) * (y - yc));
      double phi0 = 0.5 * (1.0 + tanh(2.0 * (R - r) / P->W));
      uint64_t k = (uint64_t)c;
      double cp0 = P->c0 * (1.0 + noise * orc_noise(seed, 2 * k + 1));
      double cm0 = P->c0 * (1.0 + noise * orc_noise(seed, 2 * k + 2));
      double psi0 = P->walls == WALLS_PERIODIC ? 0.0 : P->dpsi * (s->ny - 0.5 - y) / s->ny;
      double e9[9], e5[5], ei[9];
      feq(0.0, 0.0, zero_u, e9);
      for (int i = 0; i < 9; ++i) s->pop[(OF_F + i) * nc + c] = e9[i];
      heq(phi0, zero_u, e9);
      for (int i = 0; i < 9; ++i) s->pop[(OF_H + i) * nc + c] = e9[i];
      ioneq(s->qi, cp0, zero_u, ei);
      for (int i = 0; i < s->qi; ++i) s->pop[(s->op + i) * nc + c] = ei[i];
      ioneq(s->qi, cm0, zero_u, ei);
      for (int i = 0; i < s->qi; ++i) s->pop[(s->on + i) * nc + c] = ei[i];
      geq(psi0, e5);
      for (int i = 0; i < 5; ++i) s->pop[(s->og + i) * nc + c] = e5[i];
      s->jprev[c] = 0.0;
      s->jprev[nc + c] = 0.0;
    }
  s->step = 0;
}

/* Initial state from given fields [ny][nx]: every population at the
 * equilibrium of its equation (Eq. 31, 38, 45, 52 with p = 0) for the given
 * phi, concentrations, potential and velocity; (phi u)(t-1) = phi u.  Any of
 * ux, uy may be NULL for a fluid at rest. */
ORC_API void orc_init_fields(orc_state *s, const double *phi0, const double *cp0,
                             const double *cm0, const double *psi0, const double *ux0,
                             const double *uy0) {
  const orc_params *P = &s->P;
  size_t nc = s->nc;
  double rho_l = P->rho_v * P->rho_r;
  for (size_t c = 0; c < nc; ++c) {
    double u[2] = {ux0 ? ux0[c] : 0.0, uy0 ? uy0[c] : 0.0};
    double rho = phi0[c] * (rho_l - P->rho_v) + P->rho_v;
    double e9[9], e5[5], ei[9];
    feq(0.0, rho, u, e9);
    for (int i = 0; i < 9; ++i) s->pop[(OF_F + i) * nc + c] = e9[i];
    heq(phi0[c], u, e9);
    for (int i = 0; i < 9; ++i) s->pop[(OF_H + i) * nc + c] = e9[i];
    ioneq(s->qi, cp0[c], u, ei);
    for (int i = 0; i < s->qi; ++i) s->pop[(s->op + i) * nc + c] = ei[i];
    ioneq(s->qi, cm0[c], u, ei);
    for (int i = 0; i < s->qi; ++i) s->pop[(s->on + i) * nc + c] = ei[i];
    geq(psi0[c], e5);
    for (int i = 0; i < 5; ++i) s->pop[(s->og + i) * nc + c] = e5[i];
    s->jprev[c] = phi0[c] * u[0];
    s->jprev[nc + c] = phi0[c] * u[1];
  }
  s->step = 0;
}

ORC_API void orc_poisson_presolve(orc_state *s, int iters) {
  for (int k = 0; k < iters; ++k) poisson_sweep(s);
}

ORC_API void orc_step(orc_state *s, int nsteps) {
  for (int n = 0; n < nsteps; ++n) {
    for (int k = 0; k < s->P.poisson_iters; ++k) poisson_sweep(s);
    compute_moments(s);
#pragma omp parallel for schedule(static)
    for (int y = 0; y < s->ny; ++y) {
      mrt_memo mm;
    memset(mm.valid, 0, sizeof mm.valid);
      for (int x = 0; x < s->nx; ++x) collide_at(s, x, y, &mm);
    }
    stream_set(s, OF_F, 9);
    stream_set(s, OF_H, 9);
    stream_set(s, s->op, s->qi);
    stream_set(s, s->on, s->qi);
    stream_set(s, s->og, 5);
    s->step += 1;
  }
}

ORC_API long orc_get_step(const orc_state *s) { return s->step; }

/* Macroscopic fields at the current time, [NFIELD][ny][nx]. */
ORC_API void orc_fields(orc_state *s, double *out) {
  compute_moments(s);
  size_t nc = s->nc;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < s->ny; ++y)
    for (int x = 0; x < s->nx; ++x) {
      macro_t m;
      macro_at(s, x, y, &m);
      size_t c = cidx(s, x, y);
      out[FLD_PHI * nc + c] = m.phi;
      out[FLD_PSI * nc + c] = m.psi;
      out[FLD_CP * nc + c] = m.cp;
      out[FLD_CM * nc + c] = m.cm;
      out[FLD_RHOE * nc + c] = m.rhoe;
      out[FLD_UX * nc + c] = m.u[0];
      out[FLD_UY * nc + c] = m.u[1];
      out[FLD_P * nc + c] = m.p;
      out[FLD_EX * nc + c] = m.E[0];
      out[FLD_EY * nc + c] = m.E[1];
    }
}

/* Sums in row-major order: [sum phi, sum rho_e, sum (sum p), sum (sum n)]. */
ORC_API void orc_sums(orc_state *s, double *out) {
  compute_moments(s);
  double a = 0.0, b = 0.0, cP = 0.0, cQ = 0.0;
  for (size_t c = 0; c < s->nc; ++c) {
    a += s->phi[c];
    b += s->P.q * (s->sp[c] - s->sn[c]);
    cP += s->sp[c];
    cQ += s->sn[c];
  }
  out[0] = a;
  out[1] = b;
  out[2] = cP;
  out[3] = cQ;
}

/* Populations per cell: 33, or 41 with D2Q9 ions. */
ORC_API int orc_npop(const orc_state *s) { return s->npop; }

/* Raw state access: populations [npop][ny][nx] at the current time and the
 * previous phi*u [2][ny][nx]. */
ORC_API void orc_get_state(const orc_state *s, double *pop, double *jprev) {
  if (pop) memcpy(pop, s->pop, (size_t)s->npop * s->nc * sizeof(double));
  if (jprev) memcpy(jprev, s->jprev, 2 * s->nc * sizeof(double));
}

ORC_API void orc_set_state(orc_state *s, const double *pop, const double *jprev) {
  if (pop) memcpy(s->pop, pop, (size_t)s->npop * s->nc * sizeof(double));
  if (jprev) memcpy(s->jprev, jprev, 2 * s->nc * sizeof(double));
}

/* ------------------------------------------------------------------------ */
/* Pieces exposed so the tests can pin them one by one.                      */
/* ------------------------------------------------------------------------ */
ORC_API void orc_lattice(int *cx9, int *cy9, double *w9, int *cx5, int *cy5, double *w5) {
  memcpy(cx9, CX9, sizeof CX9); memcpy(cy9, CY9, sizeof CY9); memcpy(w9, W9, sizeof W9);
  memcpy(cx5, CX5, sizeof CX5); memcpy(cy5, CY5, sizeof CY5); memcpy(w5, W5, sizeof W5);
}

ORC_API int orc_matrices(double *m9, double *m9i, double *n5, double *n5i) {
  memcpy(m9, M9, sizeof M9);
  memcpy(n5, N5, sizeof N5);
  return invert(9, M9, m9i) | invert(5, N5, n5i);
}

ORC_API void orc_mrt(int q, const double *s, double *A, double *B) {
  double inv[81];
  const double *M = q == 9 ? M9 : N5;
  invert(q, M, inv);
  mrt_operators(q, M, inv, s, A, B);
}

ORC_API void orc_feq(double p, double rho, double ux, double uy, double *out) {
  double u[2] = {ux, uy};
  feq(p, rho, u, out);
}
ORC_API void orc_fforce(double ux, double uy, double grx, double gry, double Fx, double Fy,
                        double *out) {
  double u[2] = {ux, uy}, g[2] = {grx, gry}, F[2] = {Fx, Fy};
  fforce(u, g, F, out);
}
ORC_API void orc_heq(double phi, double ux, double uy, double *out) {
  double u[2] = {ux, uy};
  heq(phi, u, out);
}
ORC_API void orc_hforce(double dJx, double dJy, double nx, double ny, double phi, double W,
                        double *out) {
  double dJ[2] = {dJx, dJy}, n[2] = {nx, ny};
  hforce(dJ, n, phi, W, out);
}
ORC_API void orc_ioneq(int q, double c, double ux, double uy, double *out) {
  double u[2] = {ux, uy};
  ioneq(q, c, u, out);
}
ORC_API void orc_ionsrc(int q, double R, double c, double Fx, double Fy, int with_L,
                        double *out) {
  double F[2] = {Fx, Fy};
  ionsrc(q, R, c, F, with_L, out);
}
ORC_API void orc_iondrift(int q, double mu, double c, double gx, double gy, double *out) {
  double g[2] = {gx, gy};
  iondrift(q, mu, c, g, out);
}
ORC_API void orc_geq(double psi, double *out) { geq(psi, out); }
ORC_API void orc_unit_normal(double gx, double gy, double n_eps, double *out) {
  double g[2] = {gx, gy};
  unit_normal(g, n_eps, out);
}
ORC_API void orc_ion_solve(double cbp, double cbm, double lam0, double *cp_cm) {
  ion_solve(cbp, cbm, lam0, &cp_cm[0], &cp_cm[1]);
}

/* grad and Laplacian of an arbitrary field with the ghost rule `ghost`
 * (0 mirror, 1 odd about the wall potential). */
ORC_API void orc_stencil_field(const orc_params *p, const double *f, int ghost, double *gx,
                               double *gy, double *lap) {
  orc_state s;
  memset(&s, 0, sizeof s);
  s.P = *p;
  s.nx = p->nx;
  s.ny = p->ny;
  s.nc = (size_t)p->nx * p->ny;
  for (int y = 0; y < s.ny; ++y)
    for (int x = 0; x < s.nx; ++x) {
      double g[2], l;
      stencil(&s, f, ghost, x, y, g, &l);
      size_t c = cidx(&s, x, y);
      gx[c] = g[0];
      gy[c] = g[1];
      lap[c] = l;
    }
}
