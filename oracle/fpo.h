/*
 * fpo.h -- plain FP64 CPU oracle of the free-stream-preserving conservative
 * finite-difference scheme with reformulated upwind dissipation
 * (Su, Cai, Pan, Hu, "Reformulated dissipation for the free-stream preserving
 * of the conservative finite difference schemes on curvilinear grids").
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against the paper.  It shares no code, header, table or helper with the GPU
 * path; nothing in the product links or calls it.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark load it.
 *
 * Array layout (all host memory, float64, C order, i fastest):
 *   state  q  : [nv][Nk][Nj][Ni], N_d = n_d + 2g, nv = 5 (3D) or 4 (2D);
 *               in 2D Nk = 1.
 *   metrics   : [nmet][Nk][Nj][Ni], nmet = 10 (3D): xi_x/J, xi_y/J, xi_z/J,
 *               eta_x/J .. eta_z/J, zeta_x/J .. zeta_z/J, 1/J;
 *               nmet = 5 (2D): xi_x/J, xi_y/J, eta_x/J, eta_y/J, 1/J.
 *   coords    : [ndim][...] with extents n_d + 2(g + Y/2) (2D: two axes).
 * Boundary kinds per axis: 0 = periodic (ghost layers of q are ignored and
 * taken from the periodic image), 1 = frozen (ghost layers of q are read and
 * never changed).
 * Return values: 0 on success, -1 on invalid arguments, -2 from the metric
 * routine when the grid is folded (1/J <= 0 somewhere).
 */
#ifndef FPO_H
#define FPO_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int ndim;   /* 2 or 3 */
    int n[3];   /* interior nodes per axis (n[2] = 1 in 2D) */
    int g;      /* ghost width of state and metric arrays */
    int bc[3];  /* 0 periodic, 1 frozen */
} fpo_grid;

typedef struct {
    int recon;         /* 0: WENO5-JS, 1: fifth-order linear upwind, 2: WENO7-JS, 3: WENOCU6 */
    int Y;             /* metric order 2, 4, 6, 8 */
    int reformulated;  /* 1: the paper's method; 0: standard scheme (Q* = 0) */
    double gamma;      /* ratio of specific heats */
    double eps;        /* WENO epsilon */
    int splitting;     /* 0: local Lax-Friedrichs speeds, 1: global (Sec. 4) */
    double mu;         /* shear viscosity (0: Euler); periodic axes only */
    double prandtl;    /* Prandtl number: conductivity = mu gamma / ((gamma - 1) Pr), T = p / rho */
} fpo_scheme;

/* Boundary faces of a block (axis a, side 0 = low, 1 = high), applied to the
 * ghost layers of every non-periodic axis before each residual evaluation:
 * 0 hold (ghosts as given), 1 zeroth-order extrapolation (supersonic
 * outflow), 2 slip wall (mirror image with the normal velocity reversed,
 * normal from the metrics of the boundary node), 3 moving planar shock
 * (ghost nodes with normal . x < offset + speed t take `post`, the others
 * `pre`; conservative states).  mask[a][s], if given, has one byte per node
 * of the face (first remaining axis fastest): nodes with 0 hold. */
typedef struct {
    int kind[3][2];
    const unsigned char *mask[3][2];
    const double *nodes; /* coordinates of the state nodes (state layout, ndim arrays) */
    double pre[5], post[5];
    double normal[3];
    double offset, speed;
} fpo_bcs;

/* the ghost layers of q at time t */
int fpo_apply_bcs(const fpo_grid *gr, const fpo_bcs *bcs, const double *met, double *q, double t);
/* TVD RK3 steps from time t0 with the boundary faces applied to each stage's
 * input at the stage time (t, t + dt, t + dt/2) */
int fpo_solve_bcs(const fpo_grid *gr, const fpo_scheme *sc, const fpo_bcs *bcs, const double *met,
                  double *q, double t0, double dt, long nsteps);
/* the global Lax-Friedrichs speeds of direction d: the largest LLF speed of
 * every face of the block, per field class (u_n - c, u_n, u_n + c) */
int fpo_glf_speeds(const fpo_grid *gr, const fpo_scheme *sc, const double *met, const double *q,
                   int d, double out[3]);

/* Sec. 2.1 eqs. (JBabc),(JB) with the central derivative of eq. (metric_discret). */
int fpo_metrics(const fpo_grid *gr, int Y, const double *xyz, double *met);
/* The same quantities at selected nodes: ijk[3*p] holds (i, j, k) relative to
 * the first interior node; out[nmet*p + c]. */
int fpo_metrics_at(const fpo_grid *gr, int Y, const double *xyz, int npts,
                   const int *ijk, double *out);

/* Face fluxes F'_{i+1/2} of direction dir (Sec. 3) at every face of every
 * interior line: layout [nv][..][n_dir + 1][..] (face index f = i + 1 for
 * face i+1/2, i = -1 .. n_dir - 1), other axes interior only. */
int fpo_face_fluxes(const fpo_grid *gr, const fpo_scheme *sc, const double *met,
                    const double *q, int dir, double *flux);

/* dQ/dt = -(1/V) sum_d (F'_{i+1/2} - F'_{i-1/2}) at interior nodes; ghost
 * entries of dqdt are set to zero. */
int fpo_residual(const fpo_grid *gr, const fpo_scheme *sc, const double *met,
                 const double *q, double *dqdt);
/* The residual at selected interior nodes only: out[nv*p + v]. */
int fpo_residual_at(const fpo_grid *gr, const fpo_scheme *sc, const double *met,
                    const double *q, int npts, const int *ijk, double *out);

/* As fpo_residual_at, with the metrics of order sc->Y evaluated on the fly
 * from the coordinates xyz instead of read from a metric array. */
int fpo_residual_at_xyz(const fpo_grid *gr, const fpo_scheme *sc, const double *xyz,
                        const double *q, int npts, const int *ijk, double *out);

/* One step of the third-order TVD Runge-Kutta scheme, in place on the
 * interior of q. */
int fpo_rk3_step(const fpo_grid *gr, const fpo_scheme *sc, const double *met,
                 double *q, double dt);
int fpo_solve(const fpo_grid *gr, const fpo_scheme *sc, const double *met,
              double *q, double dt, long nsteps);

/* CFL time step: cfl / max_i sum_d (|s_d . u| + c |s_d|) / V. */
double fpo_max_dt(const fpo_grid *gr, const fpo_scheme *sc, const double *met,
                  const double *q, double cfl);

/* Building blocks exposed for the pins. */
double fpo_weno5(const double v[5], double eps);       /* eq. (weno) */
double fpo_linear_upwind5(const double v[5]);          /* eq. (linear_upwind) */
double fpo_weno7(const double v[7], double eps);       /* WENO7-JS (Remark 2) */
/* its four candidate face values q[k] and smoothness indicators beta[k] */
void fpo_weno7_parts(const double v[7], double q[4], double beta[4]);
double fpo_wenocu6(const double v[6], double eps);     /* WENOCU6 (Remark 2) */
/* its candidate face values and smoothness measures (beta[3] = beta6) */
void fpo_wenocu6_parts(const double v[6], double q[4], double beta[4]);
double fpo_face_interp(int Y, const double *w);        /* eq. (metric_discret) */
int fpo_eigensystem(int ndim, double gamma, const double *qL, const double *qR,
                    const double *sf, double Vf, double *L, double *R, double *lam);
int fpo_num_threads(void);
void fpo_set_num_threads(int n);

#ifdef __cplusplus
}
#endif

#endif /* FPO_H */
