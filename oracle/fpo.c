/*
 * fpo.c -- plain FP64 CPU oracle of the free-stream-preserving conservative
 * finite-difference scheme with reformulated upwind dissipation (Su, Cai,
 * Pan, Hu).  TEST INFRASTRUCTURE ONLY: see fpo.h.
 *
 * Every function follows the paper's definitions in the paper's order and
 * notation, one node or face at a time, with no blocking, fusion or
 * reordering.  Where the paper is silent the readings used are stated next to
 * the code (tangent basis, Roe states, local Lax-Friedrichs speeds, face
 * interpolation order, 2D metrics).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include "fpo.h"

#define NVMAX 5

/* ------------------------------------------------------------------------ */
/* array layout                                                             */
/* ------------------------------------------------------------------------ */

typedef struct {
    int ndim, nv, nmet, g;
    int n[3];   /* interior nodes (n[2] = 1 in 2D) */
    int N[3];   /* stored nodes per axis (N[2] = 1 in 2D) */
    int gk;     /* ghost offset along k (0 in 2D) */
    long vol;   /* nodes per variable */
    int bc[3];
} layout;

static int make_layout(const fpo_grid *gr, layout *L)
{
    if (!gr || (gr->ndim != 2 && gr->ndim != 3) || gr->g < 3 || gr->g > 8)
        return -1;
    L->ndim = gr->ndim;
    L->nv = gr->ndim + 2;
    L->nmet = gr->ndim == 3 ? 10 : 5;
    L->g = gr->g;
    for (int d = 0; d < 3; d++) {
        L->n[d] = gr->n[d];
        L->bc[d] = gr->bc[d];
    }
    if (gr->ndim == 2) {
        L->n[2] = 1;
        L->bc[2] = 0;
    }
    for (int d = 0; d < gr->ndim; d++) {
        if (L->n[d] < 1 || (L->bc[d] != 0 && L->bc[d] != 1))
            return -1;
        /* a periodic axis must hold at least as many nodes as one ghost layer */
        if (L->bc[d] == 0 && L->n[d] < L->g)
            return -1;
        L->N[d] = L->n[d] + 2 * L->g;
    }
    if (gr->ndim == 2) {
        L->N[2] = 1;
        L->gk = 0;
    } else {
        L->gk = L->g;
    }
    L->vol = (long)L->N[0] * L->N[1] * L->N[2];
    return 0;
}

/* offset of node (i, j, k), indices relative to the first interior node */
static long at(const layout *L, int i, int j, int k)
{
    return ((long)(k + L->gk) * L->N[1] + (j + L->g)) * L->N[0] + (i + L->g);
}

/* ------------------------------------------------------------------------ */
/* central face interpolation I_Y and derivative D_Y, eq. (metric_discret)   */
/* ------------------------------------------------------------------------ */

/* w[0 .. Y-1] hold nodes i-Y/2+1 .. i+Y/2; returns the value at face i+1/2 */
double fpo_face_interp(int Y, const double *w)
{
    switch (Y) {
    case 2:
        return (w[0] + w[1]) / 2.0;
    case 4:
        return (-w[0] + 7.0 * w[1] + 7.0 * w[2] - w[3]) / 12.0;
    case 6:
        return (w[0] - 8.0 * w[1] + 37.0 * w[2] + 37.0 * w[3] - 8.0 * w[4] + w[5]) / 60.0;
    case 8:
        return (-3.0 * w[0] + 29.0 * w[1] - 139.0 * w[2] + 533.0 * w[3] + 533.0 * w[4]
                - 139.0 * w[5] + 29.0 * w[6] - 3.0 * w[7]) / 840.0;
    }
    return NAN;
}

/* D_Y at node i from samples w[0 .. Y] = nodes i-Y/2 .. i+Y/2:
 * (x_xi)_i = x_{i+1/2} - x_{i-1/2} */
static double deriv_Y(int Y, const double *w)
{
    return fpo_face_interp(Y, w + 1) - fpo_face_interp(Y, w);
}

/* ------------------------------------------------------------------------ */
/* symmetric conservative metrics, eqs. (JBabc) and (JB)                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    const double *xyz;
    int ndim, Y, gc;
    int Nc[3];
    long volc;
} cgrid;

enum { XI = 0, ETA = 1, ZETA = 2 };
enum { CX = 0, CY = 1, CZ = 2 };

static double crd(const cgrid *C, int c, const int p[3])
{
    long off;
    if (C->ndim == 2)
        off = (long)(p[1] + C->gc) * C->Nc[0] + (p[0] + C->gc);
    else
        off = ((long)(p[2] + C->gc) * C->Nc[1] + (p[1] + C->gc)) * C->Nc[0] + (p[0] + C->gc);
    return C->xyz[c * C->volc + off];
}

/* derivative of coordinate c along computational axis e at node p */
static double dcrd(const cgrid *C, int c, int e, const int p[3])
{
    double w[9];
    int h = C->Y / 2, q[3] = {p[0], p[1], p[2]};
    for (int m = -h; m <= h; m++) {
        q[e] = p[e] + m;
        w[m + h] = crd(C, c, q);
    }
    return deriv_Y(C->Y, w);
}

/* T(a, e, b, f) = ( a_e * b )_f : derivative along f of (D_e a) times b */
static double T(const cgrid *C, int a, int e, int b, int f, const int p[3])
{
    double w[9];
    int h = C->Y / 2, q[3] = {p[0], p[1], p[2]};
    for (int m = -h; m <= h; m++) {
        q[f] = p[f] + m;
        w[m + h] = dcrd(C, a, e, q) * crd(C, b, q);
    }
    return deriv_Y(C->Y, w);
}

/* the metrics s_{d,c} = (d_c)/J of eq. (JBabc) at node p (3D) for one
 * direction d, written term by term as printed: e.g.
 * xi_x/J = 1/2[(y_eta z)_zeta - (y_zeta z)_eta + (y z_zeta)_eta - (y z_eta)_zeta] */
static void scmm3_dir(const cgrid *C, int d, const int p[3], double s[3])
{
    if (d == XI) {
        /* xi_x/J */
        s[0] = 0.5 * (T(C, CY, ETA, CZ, ZETA, p) - T(C, CY, ZETA, CZ, ETA, p)
                      + T(C, CZ, ZETA, CY, ETA, p) - T(C, CZ, ETA, CY, ZETA, p));
        /* xi_y/J = 1/2[(x z_eta)_zeta - (x z_zeta)_eta + (x_zeta z)_eta - (x_eta z)_zeta] */
        s[1] = 0.5 * (T(C, CZ, ETA, CX, ZETA, p) - T(C, CZ, ZETA, CX, ETA, p)
                      + T(C, CX, ZETA, CZ, ETA, p) - T(C, CX, ETA, CZ, ZETA, p));
        /* xi_z/J = 1/2[(x_eta y)_zeta - (x_zeta y)_eta + (x y_zeta)_eta - (x y_eta)_zeta] */
        s[2] = 0.5 * (T(C, CX, ETA, CY, ZETA, p) - T(C, CX, ZETA, CY, ETA, p)
                      + T(C, CY, ZETA, CX, ETA, p) - T(C, CY, ETA, CX, ZETA, p));
    } else if (d == ETA) {
        /* eta_x/J = 1/2[(y_zeta z)_xi - (y_xi z)_zeta + (y z_xi)_zeta - (y z_zeta)_xi] */
        s[0] = 0.5 * (T(C, CY, ZETA, CZ, XI, p) - T(C, CY, XI, CZ, ZETA, p)
                      + T(C, CZ, XI, CY, ZETA, p) - T(C, CZ, ZETA, CY, XI, p));
        /* eta_y/J = 1/2[(x z_zeta)_xi - (x z_xi)_zeta + (x_xi z)_zeta - (x_zeta z)_xi] */
        s[1] = 0.5 * (T(C, CZ, ZETA, CX, XI, p) - T(C, CZ, XI, CX, ZETA, p)
                      + T(C, CX, XI, CZ, ZETA, p) - T(C, CX, ZETA, CZ, XI, p));
        /* eta_z/J = 1/2[(x_zeta y)_xi - (x_xi y)_zeta + (x y_xi)_zeta - (x y_zeta)_xi] */
        s[2] = 0.5 * (T(C, CX, ZETA, CY, XI, p) - T(C, CX, XI, CY, ZETA, p)
                      + T(C, CY, XI, CX, ZETA, p) - T(C, CY, ZETA, CX, XI, p));
    } else {
        /* zeta_x/J = 1/2[(y_xi z)_eta - (y_eta z)_xi + (y z_eta)_xi - (y z_xi)_eta] */
        s[0] = 0.5 * (T(C, CY, XI, CZ, ETA, p) - T(C, CY, ETA, CZ, XI, p)
                      + T(C, CZ, ETA, CY, XI, p) - T(C, CZ, XI, CY, ETA, p));
        /* zeta_y/J = 1/2[(x z_xi)_eta - (x z_eta)_xi + (x_eta z)_xi - (x_xi z)_eta] */
        s[1] = 0.5 * (T(C, CZ, XI, CX, ETA, p) - T(C, CZ, ETA, CX, XI, p)
                      + T(C, CX, ETA, CZ, XI, p) - T(C, CX, XI, CZ, ETA, p));
        /* zeta_z/J = 1/2[(x_xi y)_eta - (x_eta y)_xi + (x y_eta)_xi - (x y_xi)_eta] */
        s[2] = 0.5 * (T(C, CX, XI, CY, ETA, p) - T(C, CX, ETA, CY, XI, p)
                      + T(C, CY, ETA, CX, XI, p) - T(C, CY, XI, CX, ETA, p));
    }
}

static void scmm3(const cgrid *C, const int p[3], double s[9])
{
    for (int d = 0; d < 3; d++)
        scmm3_dir(C, d, p, s + 3 * d);
}

/* 2D reduction of eq. (JBabc) (z = zeta, nothing depends on zeta):
 * xi_x/J = y_eta, xi_y/J = -x_eta, eta_x/J = -y_xi, eta_y/J = x_xi */
static void scmm2(const cgrid *C, const int p[3], double s[4])
{
    s[0] = dcrd(C, CY, ETA, p);
    s[1] = -dcrd(C, CX, ETA, p);
    s[2] = -dcrd(C, CY, XI, p);
    s[3] = dcrd(C, CX, XI, p);
}

/* 1/J of eq. (JB): 1/3 sum_d ( x s_{d,x} + y s_{d,y} + z s_{d,z} )_d (3D);
 * in 2D the same construction with z = zeta reduces to
 * 1/2 [ (x y_eta - y x_eta)_xi + (y x_xi - x y_xi)_eta ]. */
static double jacobian_inv(const cgrid *C, const int p[3])
{
    double w[9];
    int h = C->Y / 2;
    if (C->ndim == 3) {
        double sum = 0.0;
        for (int d = 0; d < 3; d++) {
            int q[3] = {p[0], p[1], p[2]};
            for (int m = -h; m <= h; m++) {
                double s[3];
                q[d] = p[d] + m;
                scmm3_dir(C, d, q, s); /* only s_d: it has no derivative along d */
                w[m + h] = crd(C, CX, q) * s[0] + crd(C, CY, q) * s[1] + crd(C, CZ, q) * s[2];
            }
            sum += deriv_Y(C->Y, w);
        }
        return sum / 3.0;
    } else {
        double a, b;
        int q[3] = {p[0], p[1], p[2]};
        for (int m = -h; m <= h; m++) {
            q[0] = p[0] + m;
            w[m + h] = crd(C, CX, q) * dcrd(C, CY, ETA, q) - crd(C, CY, q) * dcrd(C, CX, ETA, q);
        }
        a = deriv_Y(C->Y, w);
        q[0] = p[0];
        for (int m = -h; m <= h; m++) {
            q[1] = p[1] + m;
            w[m + h] = crd(C, CY, q) * dcrd(C, CX, XI, q) - crd(C, CX, q) * dcrd(C, CY, XI, q);
        }
        b = deriv_Y(C->Y, w);
        return 0.5 * (a + b);
    }
}

static void metrics_node(const cgrid *C, const int p[3], double *out /* nmet */)
{
    if (C->ndim == 3) {
        scmm3(C, p, out);
        out[9] = jacobian_inv(C, p);
    } else {
        scmm2(C, p, out);
        out[4] = jacobian_inv(C, p);
    }
}

static int make_cgrid(const layout *L, int Y, const double *xyz, cgrid *C)
{
    if (Y != 2 && Y != 4 && Y != 6 && Y != 8)
        return -1;
    if (L->g < Y / 2) /* the face interpolation I_Y reaches Y/2 nodes */
        return -1;
    C->xyz = xyz;
    C->ndim = L->ndim;
    C->Y = Y;
    C->gc = L->g + Y / 2;
    for (int d = 0; d < 3; d++)
        C->Nc[d] = d < L->ndim ? L->n[d] + 2 * C->gc : 1;
    C->volc = (long)C->Nc[0] * C->Nc[1] * C->Nc[2];
    return 0;
}

int fpo_metrics(const fpo_grid *gr, int Y, const double *xyz, double *met)
{
    layout L;
    cgrid C;
    if (make_layout(gr, &L) || make_cgrid(&L, Y, xyz, &C) || !met)
        return -1;
    int lo[3], hi[3];
    for (int d = 0; d < 3; d++) {
        if (d >= L.ndim) {
            lo[d] = 0;
            hi[d] = 1;
        } else if (L.bc[d] == 0) { /* periodic: interior, then copy to ghosts */
            lo[d] = 0;
            hi[d] = L.n[d];
        } else { /* frozen: computed on the ghost nodes from the coordinates */
            lo[d] = -L.g;
            hi[d] = L.n[d] + L.g;
        }
    }
    memset(met, 0, sizeof(double) * L.nmet * L.vol);
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = lo[2]; k < hi[2]; k++)
        for (int j = lo[1]; j < hi[1]; j++)
            for (int i = lo[0]; i < hi[0]; i++) {
                int p[3] = {i, j, k};
                double m[10];
                metrics_node(&C, p, m);
                for (int c = 0; c < L.nmet; c++)
                    met[c * L.vol + at(&L, i, j, k)] = m[c];
            }
    /* the method needs a non-degenerate, non-folded grid: 1/J > 0 */
    for (int k = lo[2]; k < hi[2]; k++)
        for (int j = lo[1]; j < hi[1]; j++)
            for (int i = lo[0]; i < hi[0]; i++)
                if (!(met[(L.nmet - 1) * L.vol + at(&L, i, j, k)] > 0.0))
                    return -2;
    /* periodic ghost layers hold exact copies of the periodic image */
    for (int d = 0; d < L.ndim; d++) {
        if (L.bc[d] != 0)
            continue;
        for (int k = (L.ndim == 3 ? -L.g : 0); k < (L.ndim == 3 ? L.n[2] + L.g : 1); k++)
            for (int j = -L.g; j < L.n[1] + L.g; j++)
                for (int i = -L.g; i < L.n[0] + L.g; i++) {
                    int p[3] = {i, j, k};
                    if (p[d] >= 0 && p[d] < L.n[d])
                        continue;
                    int src[3] = {i, j, k};
                    src[d] = ((p[d] % L.n[d]) + L.n[d]) % L.n[d];
                    for (int c = 0; c < L.nmet; c++)
                        met[c * L.vol + at(&L, i, j, k)] =
                            met[c * L.vol + at(&L, src[0], src[1], src[2])];
                }
    }
    return 0;
}

int fpo_metrics_at(const fpo_grid *gr, int Y, const double *xyz, int npts,
                   const int *ijk, double *out)
{
    layout L;
    cgrid C;
    if (make_layout(gr, &L) || make_cgrid(&L, Y, xyz, &C) || npts < 0)
        return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int t = 0; t < npts; t++) {
        int p[3] = {ijk[3 * t], ijk[3 * t + 1], L.ndim == 3 ? ijk[3 * t + 2] : 0};
        metrics_node(&C, p, out + (long)L.nmet * t);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Euler fluxes, eqs. (F)-(H) and (EOS)                                     */
/* ------------------------------------------------------------------------ */

/* pressure from the conserved state: p = (gamma-1) rho e, e = E - |u|^2/2 */
static double pressure(int ndim, double gam, const double *Q)
{
    double rho = Q[0], ke = 0.0;
    for (int c = 0; c < ndim; c++)
        ke += Q[1 + c] * Q[1 + c];
    ke = 0.5 * ke / rho;
    return (gam - 1.0) * (Q[ndim + 1] - ke);
}

/* physical fluxes F (x), G (y), H (z) of the state Q: Fx[c][v] */
static void phys_flux(int ndim, double gam, const double *Q, double Fx[3][NVMAX])
{
    int nv = ndim + 2;
    double rho = Q[0], p = pressure(ndim, gam, Q);
    for (int c = 0; c < ndim; c++) {
        double uc = Q[1 + c] / rho;
        Fx[c][0] = Q[1 + c];                       /* rho u_c */
        for (int a = 0; a < ndim; a++)             /* rho u_a u_c + p delta_ac */
            Fx[c][1 + a] = Q[1 + a] * uc + (a == c ? p : 0.0);
        Fx[c][nv - 1] = (Q[nv - 1] + p) * uc;      /* (rho E + p) u_c */
    }
}

/* ------------------------------------------------------------------------ */
/* characteristic system of A = dF~/dQ~ at the face                          */
/* ------------------------------------------------------------------------ */

/* Roe average of the two nodes adjacent to the face; eigenvectors of the
 * flux Jacobian along the unit normal n = s_f/|s_f|, eigenvalues scaled by
 * sigma = |s_f| / (1/J)_f (A acts on Q~ = Q/J).  Degenerate eigenvectors use
 * the tangent t1 = normalize(n x e_a) with a = argmin |n_k| (lowest k on
 * ties within 1e-10) and t2 = n x t1; in 2D t = (-n_y, n_x).  Field order: u_n - c,
 * u_n (entropy), tangential field(s), u_n + c. */
typedef struct {
    double R[NVMAX][NVMAX];  /* R[row][s]: column s is r_s */
    double L[NVMAX][NVMAX];  /* L[s][col]: row s is l_s */
    double lam[NVMAX];       /* Roe eigenvalues sigma*(u_n + kappa_s c) */
    double n[3];
    double sigma;
} charsys;

static void roe_system(int ndim, double gam, const double *QL, const double *QR,
                       const double *sf, double Vf, charsys *S)
{
    int nv = ndim + 2;
    double uL[3] = {0, 0, 0}, uR[3] = {0, 0, 0}, u[3] = {0, 0, 0};
    double pL = pressure(ndim, gam, QL), pR = pressure(ndim, gam, QR);
    double HL = (QL[nv - 1] + pL) / QL[0], HR = (QR[nv - 1] + pR) / QR[0];
    double wL = sqrt(QL[0]), wR = sqrt(QR[0]);
    for (int c = 0; c < ndim; c++) {
        uL[c] = QL[1 + c] / QL[0];
        uR[c] = QR[1 + c] / QR[0];
        u[c] = (wL * uL[c] + wR * uR[c]) / (wL + wR);
    }
    double H = (wL * HL + wR * HR) / (wL + wR);
    double q2 = 0.0;
    for (int c = 0; c < ndim; c++)
        q2 += u[c] * u[c];
    double cs = sqrt((gam - 1.0) * (H - 0.5 * q2));

    double snorm = 0.0;
    for (int c = 0; c < ndim; c++)
        snorm += sf[c] * sf[c];
    snorm = sqrt(snorm);
    double n[3] = {0, 0, 0};
    for (int c = 0; c < ndim; c++)
        n[c] = sf[c] / snorm;
    double un = 0.0;
    for (int c = 0; c < ndim; c++)
        un += n[c] * u[c];
    S->sigma = snorm / Vf;
    for (int c = 0; c < 3; c++)
        S->n[c] = n[c];

    double b2 = (gam - 1.0) / (cs * cs);
    double b1 = 0.5 * b2 * q2;
    memset(S->R, 0, sizeof S->R);
    memset(S->L, 0, sizeof S->L);

    int last = nv - 1;
    /* acoustic fields s = 0 (u_n - c) and s = last (u_n + c), entropy s = 1 */
    S->R[0][0] = 1.0;
    S->R[0][1] = 1.0;
    S->R[0][last] = 1.0;
    for (int c = 0; c < ndim; c++) {
        S->R[1 + c][0] = u[c] - cs * n[c];
        S->R[1 + c][1] = u[c];
        S->R[1 + c][last] = u[c] + cs * n[c];
    }
    S->R[last][0] = H - cs * un;
    S->R[last][1] = 0.5 * q2;
    S->R[last][last] = H + cs * un;

    S->L[0][0] = 0.5 * (b1 + un / cs);
    S->L[1][0] = 1.0 - b1;
    S->L[last][0] = 0.5 * (b1 - un / cs);
    for (int c = 0; c < ndim; c++) {
        S->L[0][1 + c] = 0.5 * (-b2 * u[c] - n[c] / cs);
        S->L[1][1 + c] = b2 * u[c];
        S->L[last][1 + c] = 0.5 * (-b2 * u[c] + n[c] / cs);
    }
    S->L[0][last] = 0.5 * b2;
    S->L[1][last] = -b2;
    S->L[last][last] = 0.5 * b2;

    /* tangential (shear) fields */
    double t[2][3];
    int nt;
    if (ndim == 2) {
        t[0][0] = -n[1];
        t[0][1] = n[0];
        t[0][2] = 0.0;
        nt = 1;
    } else {
        /* components closer than 1e-10 count as tied (lowest k wins), so
         * that grids with a symmetric normal do not depend on rounding */
        int a = 0;
        for (int c = 1; c < 3; c++)
            if (fabs(n[c]) < fabs(n[a]) - 1e-10)
                a = c;
        double e[3] = {0, 0, 0};
        e[a] = 1.0;
        double x[3] = {n[1] * e[2] - n[2] * e[1], n[2] * e[0] - n[0] * e[2],
                       n[0] * e[1] - n[1] * e[0]};
        double xn = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        for (int c = 0; c < 3; c++)
            t[0][c] = x[c] / xn;
        t[1][0] = n[1] * t[0][2] - n[2] * t[0][1];
        t[1][1] = n[2] * t[0][0] - n[0] * t[0][2];
        t[1][2] = n[0] * t[0][1] - n[1] * t[0][0];
        nt = 2;
    }
    for (int r = 0; r < nt; r++) {
        int s = 2 + r;
        double ut = 0.0;
        for (int c = 0; c < ndim; c++)
            ut += u[c] * t[r][c];
        S->R[0][s] = 0.0;
        for (int c = 0; c < ndim; c++)
            S->R[1 + c][s] = t[r][c];
        S->R[last][s] = ut;
        S->L[s][0] = -ut;
        for (int c = 0; c < ndim; c++)
            S->L[s][1 + c] = t[r][c];
        S->L[s][last] = 0.0;
    }
    for (int s = 0; s < nv; s++) {
        double kap = s == 0 ? -1.0 : (s == last ? 1.0 : 0.0);
        S->lam[s] = S->sigma * (un + kap * cs);
    }
}

int fpo_eigensystem(int ndim, double gamma, const double *qL, const double *qR,
                    const double *sf, double Vf, double *Lout, double *Rout, double *lam)
{
    if (ndim != 2 && ndim != 3)
        return -1;
    charsys S;
    int nv = ndim + 2;
    roe_system(ndim, gamma, qL, qR, sf, Vf, &S);
    for (int a = 0; a < nv; a++) {
        for (int b = 0; b < nv; b++) {
            Lout[a * nv + b] = S.L[a][b];
            Rout[a * nv + b] = S.R[a][b];
        }
        lam[a] = S.lam[a];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* reconstructions                                                          */
/* ------------------------------------------------------------------------ */

/* WENO5-JS, eq. (weno) with eq. (weno_wights); v = (f_{i-2} .. f_{i+2}).
 * Readings: q0 = f_{i-2}/3 - 7 f_{i-1}/6 + 11 f_i/6 (the printed 7/6 on f_i
 * breaks consistency), and the weight denominator sums C_r/(beta_r+eps)^2. */
double fpo_weno5(const double v[5], double eps)
{
    const double C[3] = {1.0 / 10.0, 3.0 / 5.0, 3.0 / 10.0};
    double q[3], beta[3], alpha[3], asum = 0.0, out = 0.0;
    q[0] = v[0] / 3.0 - 7.0 * v[1] / 6.0 + 11.0 * v[2] / 6.0;
    q[1] = -v[1] / 6.0 + 5.0 * v[2] / 6.0 + v[3] / 3.0;
    q[2] = v[2] / 3.0 + 5.0 * v[3] / 6.0 - v[4] / 6.0;
    beta[0] = 0.25 * pow(v[0] - 4.0 * v[1] + 3.0 * v[2], 2)
              + 13.0 / 12.0 * pow(v[0] - 2.0 * v[1] + v[2], 2);
    beta[1] = 0.25 * pow(-v[1] + v[3], 2) + 13.0 / 12.0 * pow(v[1] - 2.0 * v[2] + v[3], 2);
    beta[2] = 0.25 * pow(-3.0 * v[2] + 4.0 * v[3] - v[4], 2)
              + 13.0 / 12.0 * pow(v[2] - 2.0 * v[3] + v[4], 2);
    for (int k = 0; k < 3; k++) {
        alpha[k] = C[k] / pow(beta[k] + eps, 2);
        asum += alpha[k];
    }
    for (int k = 0; k < 3; k++)
        out += alpha[k] / asum * q[k];
    return out;
}

/* fifth-order linear upwind, eq. (linear_upwind), "+" orientation */
double fpo_linear_upwind5(const double v[5])
{
    return (2.0 * v[0] - 13.0 * v[1] + 47.0 * v[2] + 27.0 * v[3] - 3.0 * v[4]) / 60.0;
}

/* WENO7-JS (the standard seventh-order WENO the paper extends its method to,
 * Remark 2): v = (f_{i-3} .. f_{i+3}), four third-degree candidates on
 * {i-3..i}, {i-2..i+1}, {i-1..i+2}, {i..i+3}, optimal weights
 * (1, 12, 18, 4)/35, and smoothness indicators that are the integer
 * quadratic forms equal to 240 x the Jiang-Shu measure
 * sum_{l=1}^{3} int_cell (d^l p_k / dx^l)^2 dx (unit spacing).  Reading:
 * the forms are used without the 1/240 (with eps = 1e-6 this reproduces the
 * WENO7 rows of Table 2; the normalised measure does not).  The weights are
 * C_k / (beta_k + eps)^2 as for WENO5. */
void fpo_weno7_parts(const double v[7], double q[4], double beta[4])
{
    const double a = v[0], b = v[1], c = v[2], d = v[3], e = v[4], f = v[5], g = v[6];
    q[0] = (-3.0 * a + 13.0 * b - 23.0 * c + 25.0 * d) / 12.0;
    q[1] = (b - 5.0 * c + 13.0 * d + 3.0 * e) / 12.0;
    q[2] = (-c + 7.0 * d + 7.0 * e - f) / 12.0;
    q[3] = (3.0 * d + 13.0 * e - 5.0 * f + g) / 12.0;
    beta[0] = (a * (547.0 * a - 3882.0 * b + 4642.0 * c - 1854.0 * d)
               + b * (7043.0 * b - 17246.0 * c + 7042.0 * d)
               + c * (11003.0 * c - 9402.0 * d) + 2107.0 * d * d);
    beta[1] = (b * (267.0 * b - 1642.0 * c + 1602.0 * d - 494.0 * e)
               + c * (2843.0 * c - 5966.0 * d + 1922.0 * e)
               + d * (3443.0 * d - 2522.0 * e) + 547.0 * e * e);
    beta[2] = (c * (547.0 * c - 2522.0 * d + 1922.0 * e - 494.0 * f)
               + d * (3443.0 * d - 5966.0 * e + 1602.0 * f)
               + e * (2843.0 * e - 1642.0 * f) + 267.0 * f * f);
    beta[3] = (d * (2107.0 * d - 9402.0 * e + 7042.0 * f - 1854.0 * g)
               + e * (11003.0 * e - 17246.0 * f + 4642.0 * g)
               + f * (7043.0 * f - 3882.0 * g) + 547.0 * g * g);
}

double fpo_weno7(const double v[7], double eps)
{
    const double C[4] = {1.0 / 35.0, 12.0 / 35.0, 18.0 / 35.0, 4.0 / 35.0};
    double q[4], beta[4], alpha[4], asum = 0.0, out = 0.0;
    fpo_weno7_parts(v, q, beta);
    for (int k = 0; k < 4; k++) {
        alpha[k] = C[k] / pow(beta[k] + eps, 2);
        asum += alpha[k];
    }
    for (int k = 0; k < 4; k++)
        out += alpha[k] / asum * q[k];
    return out;
}

/* The polynomial p(x) = sum_k c[k] x^k of degree n-1 whose averages over the
 * unit cells [m-1/2, m+1/2], m = m0 .. m0+n-1, are f[0..n-1] (x measured from
 * the centre of the cell left of the face, unit spacing): the cell-average
 * reconstruction behind every WENO candidate.  The averaging matrix
 * A[r][k] = ((m0+r+1/2)^(k+1) - (m0+r-1/2)^(k+1))/(k+1) depends only on the
 * stencil, so its inverse is formed once per stencil (Gauss-Jordan with
 * partial pivoting) and each reconstruction is c = A^-1 f. */
static void invert_avg(int n, int m0, double inv[6][6])
{
    double A[6][12];
    for (int r = 0; r < n; r++) {
        double lo = m0 + r - 0.5, hi = m0 + r + 0.5;
        for (int k = 0; k < n; k++) {
            A[r][k] = (pow(hi, k + 1) - pow(lo, k + 1)) / (k + 1);
            A[r][n + k] = r == k ? 1.0 : 0.0;
        }
    }
    for (int col = 0; col < n; col++) {
        int piv = col;
        for (int r = col + 1; r < n; r++)
            if (fabs(A[r][col]) > fabs(A[piv][col]))
                piv = r;
        for (int k = 0; k < 2 * n; k++) {
            double t = A[col][k];
            A[col][k] = A[piv][k];
            A[piv][k] = t;
        }
        double d = A[col][col];
        for (int k = 0; k < 2 * n; k++)
            A[col][k] /= d;
        for (int r = 0; r < n; r++) {
            if (r == col)
                continue;
            double fac = A[r][col];
            for (int k = 0; k < 2 * n; k++)
                A[r][k] -= fac * A[col][k];
        }
    }
    for (int r = 0; r < n; r++)
        for (int k = 0; k < n; k++)
            inv[r][k] = A[r][n + k];
}

/* the inverses of the four quadratic candidates' stencils {k-2 .. k}
 * (relative to cell i) and of the quintic's {-2 .. 3}; formed on first use */
static double g_inv3[4][6][6], g_inv6[6][6];
static int g_inv_ready = 0;

static void cu6_tables(void)
{
#pragma omp critical(fpo_cu6_tables)
    if (!g_inv_ready) {
        for (int k = 0; k < 4; k++)
            invert_avg(3, k - 2, g_inv3[k]);
        invert_avg(6, -2, g_inv6);
        g_inv_ready = 1;
    }
}

static void cellavg_poly(int n, const double inv[6][6], const double *f, double *c)
{
    for (int k = 0; k < n; k++) {
        double s = 0.0;
        for (int r = 0; r < n; r++)
            s += inv[k][r] * f[r];
        c[k] = s;
    }
}

static double poly_at(int n, const double *c, double x)
{
    double s = 0.0;
    for (int k = n - 1; k >= 0; k--)
        s = s * x + c[k];
    return s;
}

/* int_{-1/2}^{1/2} x^e dx */
static double mono_int(int e)
{
    return (e % 2) ? 0.0 : 1.0 / ((e + 1) * (double)(1L << e));
}

/* smoothness of a candidate in the Jiang-Shu sense at unit spacing:
 * sum_{l=1}^{n-1} int_{-1/2}^{1/2} (p^(l)(x))^2 dx over the cell left of the
 * face */
static double smoothness(int n, const double *c)
{
    double d[6], tot = 0.0;
    for (int k = 0; k < n; k++)
        d[k] = c[k];
    for (int l = 1; l < n; l++) {
        int m = n - l; /* terms of the l-th derivative */
        for (int k = 0; k < m; k++)
            d[k] = (k + 1) * d[k + 1];
        for (int a = 0; a < m; a++)
            for (int b = 0; b < m; b++)
                tot += d[a] * d[b] * mono_int(a + b);
    }
    return tot;
}

/* WENOCU6, the sixth-order adaptive central-upwind WENO the paper extends its
 * method to (Remark 2; Hu, Wang and Adams 2010): v = (f_{i-2} .. f_{i+3}),
 * the face i+1/2.  Candidates: the quadratic cell-average reconstructions on
 * {i-2..i}, {i-1..i+1}, {i..i+2} and the downwind {i+1..i+3}, evaluated at the
 * face; optimal weights (1, 9, 9, 1)/20 (together the sixth-order central
 * interpolation).  Smoothness: the Jiang-Shu measure of the three upwind
 * candidates, and for the downwind slot the measure beta6 of the quintic
 * reconstruction over all six cells, both integrated over cell i.  Weights
 * alpha_k = d_k (C + tau6/(beta_k + eps))^q with
 * tau6 = beta6 - (beta_0 + 4 beta_1 + beta_2)/6, C = 20, q = 2 (the cited
 * scheme's constants; the paper gives none) and the caller's eps (the paper's
 * WENO epsilon, 1e-6).  Everything here comes from the definitions:
 * reconstruct, evaluate, integrate. */
/* (the tables must be formed: check_scheme and the public entry points do
 * it before any parallel region) */
static void wenocu6_parts(const double v[6], double q[4], double beta[4])
{
    double c[6];
    for (int k = 0; k < 4; k++) {
        cellavg_poly(3, g_inv3[k], v + k, c);
        q[k] = poly_at(3, c, 0.5);
        beta[k] = smoothness(3, c);
    }
    cellavg_poly(6, g_inv6, v, c);
    beta[3] = smoothness(6, c);
}

void fpo_wenocu6_parts(const double v[6], double q[4], double beta[4])
{
    cu6_tables();
    wenocu6_parts(v, q, beta);
}

static double wenocu6(const double v[6], double eps)
{
    const double d[4] = {1.0 / 20.0, 9.0 / 20.0, 9.0 / 20.0, 1.0 / 20.0};
    const double C = 20.0, qexp = 2.0;
    double q[4], beta[4], alpha[4], asum = 0.0, out = 0.0;
    wenocu6_parts(v, q, beta);
    double tau6 = beta[3] - (beta[0] + 4.0 * beta[1] + beta[2]) / 6.0;
    for (int k = 0; k < 4; k++) {
        alpha[k] = d[k] * pow(C + tau6 / (beta[k] + eps), qexp);
        asum += alpha[k];
    }
    for (int k = 0; k < 4; k++)
        out += alpha[k] / asum * q[k];
    return out;
}

double fpo_wenocu6(const double v[6], double eps)
{
    cu6_tables();
    return wenocu6(v, eps);
}

/* half-width of the split-flux stencil below the face node i: the "+" part
 * uses f_{i-lo} .. f_{i+lo} (WENOCU6: .. f_{i+lo+1}), the "-" part
 * f_{i+lo+1} .. f_{i-lo+1} (WENOCU6: .. f_{i-lo}) */
static int stencil_lo(const fpo_scheme *sc)
{
    return sc->recon == 2 ? 3 : 2;
}

/* values a reconstruction takes from the split-flux stencil of 2 lo + 2 */
static int recon_width(const fpo_scheme *sc)
{
    return sc->recon == 3 ? 2 * stencil_lo(sc) + 2 : 2 * stencil_lo(sc) + 1;
}

static double reconstruct(const fpo_scheme *sc, const double *v)
{
    if (sc->recon == 3)
        return wenocu6(v, sc->eps);
    if (sc->recon == 2)
        return fpo_weno7(v, sc->eps);
    return sc->recon == 1 ? fpo_linear_upwind5(v) : fpo_weno5(v, sc->eps);
}

/* ------------------------------------------------------------------------ */
/* face flux with the reformulated dissipation (Sec. 3)                      */
/* ------------------------------------------------------------------------ */

typedef struct {
    int ndim, nv;
    const double *Q[NVMAX]; /* Q[v][m], m relative to the first interior node */
    const double *V;        /* 1/J */
    const double *S[3];     /* metric vector of the sweep direction, s_{d,c} */
} line_t;

/* local Lax-Friedrichs speed of every field at the face i+1/2 with unit
 * normal n and metric norm sigma: the largest sigma |n . u_m + kappa_s c_m|
 * over the stencil m = i-lo .. i+lo+1 */
static void llf_speeds(const fpo_scheme *sc, const line_t *ln, int i, const double *n, double sigma,
                       double *lam)
{
    const int ndim = ln->ndim, nv = ln->nv, lo = stencil_lo(sc), ns = 2 * lo + 2;
    for (int s = 0; s < nv; s++) {
        double kap = s == 0 ? -1.0 : (s == nv - 1 ? 1.0 : 0.0);
        lam[s] = 0.0;
        for (int r = 0; r < ns; r++) {
            int m = i - lo + r;
            double Qm[NVMAX];
            for (int v = 0; v < nv; v++)
                Qm[v] = ln->Q[v][m];
            double unm = 0.0;
            for (int c = 0; c < ndim; c++)
                unm += n[c] * Qm[1 + c] / Qm[0];
            double cm = sqrt(sc->gamma * pressure(ndim, sc->gamma, Qm) / Qm[0]);
            double a = sigma * fabs(unm + kap * cm);
            if (a > lam[s])
                lam[s] = a;
        }
    }
}

/* F'_{i+1/2} for the face between nodes i and i+1 of a line; glf = NULL
 * for local Lax-Friedrichs speeds, else the block's global speeds of the
 * three field classes (u_n - c, u_n, u_n + c) */
static void face_flux(const fpo_scheme *sc, const line_t *ln, int i, const double *glf, double *Fp)
{
    const int ndim = ln->ndim, nv = ln->nv, Y = sc->Y, h = Y / 2;
    const double gam = sc->gamma;
    double w[8];

    /* (1) cell-face reference state: (1/J)_{i+1/2}, Q~_{i+1/2} and the face
     * metrics by the central interpolation of the metric order Y
     * (eqs. QdJ_star, 1dJ, xidJ; Remark 3 asks for the metric scheme), and
     * Q* = Q~_{i+1/2} / (1/J)_{i+1/2} (eq. Q_star). */
    double Vf, Qtf[NVMAX], sf[3] = {0, 0, 0}, Qs[NVMAX];
    for (int m = 0; m < Y; m++)
        w[m] = ln->V[i - h + 1 + m];
    Vf = fpo_face_interp(Y, w);
    for (int v = 0; v < nv; v++) {
        for (int m = 0; m < Y; m++)
            w[m] = ln->Q[v][i - h + 1 + m] * ln->V[i - h + 1 + m];
        Qtf[v] = fpo_face_interp(Y, w);
    }
    for (int c = 0; c < ndim; c++) {
        for (int m = 0; m < Y; m++)
            w[m] = ln->S[c][i - h + 1 + m];
        sf[c] = fpo_face_interp(Y, w);
    }
    for (int v = 0; v < nv; v++)
        Qs[v] = sc->reformulated ? Qtf[v] / Vf : 0.0;

    /* (2) fluxes F*, G*, H* of Q* and the face flux
     * F~*_{i+1/2} = F* (xi_x/J)_{i+1/2} + G* (xi_y/J)_{i+1/2} + H* (xi_z/J)_{i+1/2} */
    double Fs[3][NVMAX], Fts[NVMAX];
    memset(Fs, 0, sizeof Fs);
    if (sc->reformulated)
        phys_flux(ndim, gam, Qs, Fs);
    for (int v = 0; v < nv; v++) {
        Fts[v] = 0.0;
        for (int c = 0; c < ndim; c++)
            Fts[v] += Fs[c][v] * sf[c];
    }

    /* (3) reference-subtracted stencil values, m = i-lo .. i+lo+1 (lo = 2 for
     * the fifth-order schemes, 3 for WENO7):
     * dQ~_m = (Q_m - Q*)/J_m and
     * dF~_m = (F_m - F*) (xi_x/J)_m + (G_m - G*) (xi_y/J)_m + (H_m - H*) (xi_z/J)_m
     * (eqs. Linear_upwind_LFspliting and flux_split_detail) */
    const int lo = stencil_lo(sc), ns = 2 * lo + 2;
    double dQt[8][NVMAX], dFt[8][NVMAX];
    for (int r = 0; r < ns; r++) {
        int m = i - lo + r;
        double Qm[NVMAX], Fm[3][NVMAX];
        for (int v = 0; v < nv; v++)
            Qm[v] = ln->Q[v][m];
        phys_flux(ndim, gam, Qm, Fm);
        for (int v = 0; v < nv; v++) {
            dQt[r][v] = (Qm[v] - Qs[v]) * ln->V[m];
            dFt[r][v] = 0.0;
            for (int c = 0; c < ndim; c++)
                dFt[r][v] += (Fm[c][v] - Fs[c][v]) * ln->S[c][m];
        }
    }

    /* (4) Roe-averaged characteristic system at i+1/2 */
    double QL[NVMAX], QR[NVMAX];
    for (int v = 0; v < nv; v++) {
        QL[v] = ln->Q[v][i];
        QR[v] = ln->Q[v][i + 1];
    }
    charsys S;
    roe_system(ndim, gam, QL, QR, sf, Vf, &S);

    /* (5) Lax-Friedrichs speed of every field: local (the largest
     * sigma |n . u_m + kappa_s c_m| over the stencil) or global (the
     * largest over every face of the block, computed beforehand) */
    double lam[NVMAX];
    if (glf) {
        for (int s = 0; s < nv; s++)
            lam[s] = s == 0 ? glf[0] : (s == nv - 1 ? glf[2] : glf[1]);
    } else {
        llf_speeds(sc, ln, i, S.n, S.sigma, lam);
    }

    /* (6) characteristic projection and Lax-Friedrichs splitting:
     * F~^{s,+-}_m = 1/2 l_s . (dF~_m +- lambda_s dQ~_m) */
    double vp[NVMAX][8], vm[NVMAX][8];
    for (int s = 0; s < nv; s++)
        for (int r = 0; r < ns; r++) {
            double a = 0.0, b = 0.0;
            for (int v = 0; v < nv; v++) {
                a += S.L[s][v] * dFt[r][v];
                b += S.L[s][v] * dQt[r][v];
            }
            vp[s][r] = 0.5 * (a + lam[s] * b);
            vm[s][r] = 0.5 * (a - lam[s] * b);
        }

    /* (7) reconstruction of both split parts at the face: the "+" part from
     * m = i-lo .. i+lo, the "-" part mirrored from m = i+lo+1 .. i-lo+1
     * (WENOCU6 takes the whole stencil in both orientations) */
    double hp[NVMAX], hm[NVMAX];
    const int nr = recon_width(sc);
    for (int s = 0; s < nv; s++) {
        double a[8], b[8];
        for (int r = 0; r < nr; r++) {
            a[r] = vp[s][r];
            b[r] = vm[s][ns - 1 - r];
        }
        hp[s] = reconstruct(sc, a);
        hm[s] = reconstruct(sc, b);
    }

    /* (8) back to physical space and add the reference flux back
     * (eq. my_point1): F'_{i+1/2} = F~*_{i+1/2} + sum_s r_s (h+_s + h-_s) */
    for (int v = 0; v < nv; v++) {
        double sum = 0.0;
        for (int s = 0; s < nv; s++)
            sum += S.R[v][s] * (hp[s] + hm[s]);
        Fp[v] = Fts[v] + sum;
    }
}

/* ------------------------------------------------------------------------ */
/* ghost layers, lines, residual                                            */
/* ------------------------------------------------------------------------ */

/* copy of q with periodic ghost layers taken from the periodic image */
static double *filled_copy(const layout *L, const double *q)
{
    double *w = (double *)malloc(sizeof(double) * L->nv * L->vol);
    if (!w)
        return NULL;
    memcpy(w, q, sizeof(double) * L->nv * L->vol);
    for (int d = 0; d < L->ndim; d++) {
        if (L->bc[d] != 0)
            continue;
        for (int k = (L->ndim == 3 ? -L->g : 0); k < (L->ndim == 3 ? L->n[2] + L->g : 1); k++)
            for (int j = -L->g; j < L->n[1] + L->g; j++)
                for (int i = -L->g; i < L->n[0] + L->g; i++) {
                    int p[3] = {i, j, k};
                    if (p[d] >= 0 && p[d] < L->n[d])
                        continue;
                    int s[3] = {i, j, k};
                    s[d] = ((p[d] % L->n[d]) + L->n[d]) % L->n[d];
                    for (int v = 0; v < L->nv; v++)
                        w[v * L->vol + at(L, i, j, k)] = w[v * L->vol + at(L, s[0], s[1], s[2])];
                }
    }
    return w;
}

/* gather the line through (p with p[d] free) into buf; fills ln */
static void gather_line(const layout *L, const double *q, const double *met, int d,
                        const int p[3], double *buf, line_t *ln)
{
    int len = L->n[d] + 2 * L->g;
    int nsd = L->ndim; /* metric components per direction */
    ln->ndim = L->ndim;
    ln->nv = L->nv;
    for (int t = 0; t < len; t++) {
        int c3[3] = {p[0], p[1], p[2]};
        c3[d] = t - L->g;
        long off = at(L, c3[0], c3[1], c3[2]);
        for (int v = 0; v < L->nv; v++)
            buf[v * len + t] = q[v * L->vol + off];
        buf[L->nv * len + t] = met[(L->nmet - 1) * L->vol + off];
        for (int c = 0; c < nsd; c++)
            buf[(L->nv + 1 + c) * len + t] = met[(d * nsd + c) * L->vol + off];
    }
    for (int v = 0; v < L->nv; v++)
        ln->Q[v] = buf + v * len + L->g;
    ln->V = buf + L->nv * len + L->g;
    for (int c = 0; c < nsd; c++)
        ln->S[c] = buf + (L->nv + 1 + c) * len + L->g;
}

static int check_scheme(const layout *L, const fpo_scheme *sc)
{
    if (!sc || sc->recon < 0 || sc->recon > 3 || (sc->reformulated != 0 && sc->reformulated != 1))
        return -1;
    if (sc->Y != 2 && sc->Y != 4 && sc->Y != 6 && sc->Y != 8)
        return -1;
    /* the split-flux stencil reaches lo + 1 nodes from a node (3 for the
     * fifth-order schemes, 4 for WENO7); the face interpolation Y/2 nodes */
    if (L->g < stencil_lo(sc) + 1 || L->g < sc->Y / 2)
        return -1;
    if (!(sc->gamma > 1.0) || !(sc->eps > 0.0) || (sc->splitting != 0 && sc->splitting != 1))
        return -1;
    if (sc->recon == 3)
        cu6_tables();
    if (sc->mu < 0.0 || (sc->mu > 0.0 && !(sc->prandtl > 0.0)))
        return -1;
    if (sc->mu > 0.0)
        for (int d = 0; d < L->ndim; d++)
            if (L->bc[d] != 0 || L->n[d] < 7)
                return -1; /* the viscous stencils wrap periodically */
    return 0;
}

/* the two axes other than d */
static void other_axes(int d, int *a, int *b)
{
    *a = d == 0 ? 1 : 0;
    *b = d == 2 ? 1 : 2;
}

/* unit normal and metric norm of the face i+1/2: the face metrics and 1/J
 * interpolated as in step (1) of the face flux, n = s_f/|s_f| and
 * sigma = |s_f|/(1/J)_f as in the Roe system of step (4) */
static void face_normal(const fpo_scheme *sc, const line_t *ln, int i, double n[3], double *sigma)
{
    const int Y = sc->Y, h = Y / 2, ndim = ln->ndim;
    double w[8], sf[3] = {0, 0, 0};
    for (int m = 0; m < Y; m++)
        w[m] = ln->V[i - h + 1 + m];
    double Vf = fpo_face_interp(Y, w);
    for (int c = 0; c < ndim; c++) {
        for (int m = 0; m < Y; m++)
            w[m] = ln->S[c][i - h + 1 + m];
        sf[c] = fpo_face_interp(Y, w);
    }
    double snorm = 0.0;
    for (int c = 0; c < ndim; c++)
        snorm += sf[c] * sf[c];
    snorm = sqrt(snorm);
    n[0] = n[1] = n[2] = 0.0;
    for (int c = 0; c < ndim; c++)
        n[c] = sf[c] / snorm;
    *sigma = snorm / Vf;
}

/* global Lax-Friedrichs speeds of direction d: the local speeds of every
 * face of the block (faces i+1/2, i = -1 .. n-1, of every interior line),
 * maximised per field class */
static void glf_filled(const layout *L, const fpo_scheme *sc, const double *met, const double *qf,
                       int d, double out[3])
{
    int a, b;
    other_axes(d, &a, &b);
    int len = L->n[d] + 2 * L->g;
    int na = L->n[a], nb = L->n[b];
    out[0] = out[1] = out[2] = 0.0;
#pragma omp parallel
    {
        double *buf = (double *)malloc(sizeof(double) * len * (L->nv + 1 + L->ndim));
        double mx[3] = {0.0, 0.0, 0.0};
        line_t ln;
#pragma omp for collapse(2) schedule(static)
        for (int ib = 0; ib < nb; ib++)
            for (int ia = 0; ia < na; ia++) {
                int p[3] = {0, 0, 0};
                p[a] = ia;
                p[b] = ib;
                gather_line(L, qf, met, d, p, buf, &ln);
                for (int f = 0; f <= L->n[d]; f++) {
                    double n[3], sigma, lam[NVMAX];
                    face_normal(sc, &ln, f - 1, n, &sigma);
                    llf_speeds(sc, &ln, f - 1, n, sigma, lam);
                    mx[0] = fmax(mx[0], lam[0]);
                    mx[1] = fmax(mx[1], lam[1]);
                    mx[2] = fmax(mx[2], lam[L->nv - 1]);
                }
            }
#pragma omp critical
        for (int k = 0; k < 3; k++)
            out[k] = fmax(out[k], mx[k]);
        free(buf);
    }
}

int fpo_glf_speeds(const fpo_grid *gr, const fpo_scheme *sc, const double *met, const double *q,
                   int d, double out[3])
{
    layout L;
    if (make_layout(gr, &L) || check_scheme(&L, sc) || d < 0 || d >= L.ndim)
        return -1;
    double *qf = filled_copy(&L, q);
    if (!qf)
        return -1;
    glf_filled(&L, sc, met, qf, d, out);
    free(qf);
    return 0;
}

int fpo_face_fluxes(const fpo_grid *gr, const fpo_scheme *sc, const double *met,
                    const double *q, int dir, double *flux)
{
    layout L;
    if (make_layout(gr, &L) || check_scheme(&L, sc) || dir < 0 || dir >= L.ndim)
        return -1;
    double *qf = filled_copy(&L, q);
    if (!qf)
        return -1;
    int a, b;
    other_axes(dir, &a, &b);
    int nf = L.n[dir] + 1;
    int ext[3] = {L.n[0], L.n[1], L.n[2]};
    ext[dir] = nf;
    long fvol = (long)ext[0] * ext[1] * ext[2];
    int na = L.n[a], nb = L.n[b];
    int len = L.n[dir] + 2 * L.g;
    double glf[3], *gp = NULL;
    if (sc->splitting) {
        glf_filled(&L, sc, met, qf, dir, glf);
        gp = glf;
    }
#pragma omp parallel
    {
        double *buf = (double *)malloc(sizeof(double) * len * (L.nv + 1 + L.ndim));
        line_t ln;
#pragma omp for collapse(2) schedule(static)
        for (int ib = 0; ib < nb; ib++)
            for (int ia = 0; ia < na; ia++) {
                int p[3] = {0, 0, 0};
                p[a] = ia;
                p[b] = ib;
                gather_line(&L, qf, met, dir, p, buf, &ln);
                for (int f = 0; f < nf; f++) {
                    double F[NVMAX];
                    face_flux(sc, &ln, f - 1, gp, F);
                    int c3[3] = {p[0], p[1], p[2]};
                    c3[dir] = f;
                    long off = ((long)c3[2] * ext[1] + c3[1]) * ext[0] + c3[0];
                    for (int v = 0; v < L.nv; v++)
                        flux[v * fvol + off] = F[v];
                }
            }
        free(buf);
    }
    free(qf);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* viscous fluxes (Sec. 2.1 eqs. NSv1-NSv3, stress, strain, heat flux;      */
/* sixth-order central differences as Sec. 2.2 states), periodic axes       */
/* ------------------------------------------------------------------------ */

/* sixth-order central first derivative, offsets -3 .. 3 */
static const double D6[7] = {-1.0 / 60.0, 9.0 / 60.0, -45.0 / 60.0, 0.0, 45.0 / 60.0, -9.0 / 60.0, 1.0 / 60.0};

/* interior node p shifted by `off` along axis d, wrapped periodically */
static long wrap_at(const layout *L, const int p[3], int d, int off)
{
    int c[3] = {p[0], p[1], p[2]};
    c[d] = ((c[d] + off) % L->n[d] + L->n[d]) % L->n[d];
    return at(L, c[0], c[1], c[2]);
}

/* acc -= sum_d D6_d(Fv~_d) at every interior node, where
 * Fv~_d = sum_j s_{d,j} Fv_j (eq. FGH_v) and, with T = p/rho,
 * tau_ij = mu (du_i/dx_j + du_j/dx_i - 2/3 delta_ij div u),
 * Fv_j = (0, tau_1j, .., tau_nj, u_i tau_ij + k dT/dx_j), k = mu gamma/((gamma-1) Pr),
 * and the gradients at a node by the chain rule
 * dphi/dx_j = (1/V) sum_d s_{d,j} D6_d(phi). */
static int viscous_acc(const layout *L, const fpo_scheme *sc, const double *met, const double *q,
                       double *acc)
{
    const int nd = L->ndim, nv = L->nv, np = nd + 1; /* primitives u_1..u_nd, T */
    const long vol = L->vol;
    const double gam = sc->gamma, mu = sc->mu;
    const double kappa = mu * gam / ((gam - 1.0) * sc->prandtl);
    double *prim = (double *)calloc((size_t)np * vol, sizeof(double));
    double *fv = (double *)calloc((size_t)nd * nv * vol, sizeof(double));
    if (!prim || !fv) {
        free(prim);
        free(fv);
        return -1;
    }
    for (int k = 0; k < L->n[2]; k++)
        for (int j = 0; j < L->n[1]; j++)
            for (int i = 0; i < L->n[0]; i++) {
                long o = at(L, i, j, k);
                double Q[NVMAX];
                for (int v = 0; v < nv; v++)
                    Q[v] = q[v * vol + o];
                for (int c = 0; c < nd; c++)
                    prim[c * vol + o] = Q[1 + c] / Q[0];
                prim[nd * vol + o] = pressure(nd, gam, Q) / Q[0];
            }
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < L->n[2]; k++)
        for (int j = 0; j < L->n[1]; j++)
            for (int i = 0; i < L->n[0]; i++) {
                int p[3] = {i, j, k};
                long o = at(L, i, j, k);
                double V = met[(L->nmet - 1) * vol + o];
                /* grad[a][jj] = d prim_a / d x_jj */
                double grad[4][3];
                for (int a = 0; a < np; a++)
                    for (int jj = 0; jj < nd; jj++)
                        grad[a][jj] = 0.0;
                for (int d = 0; d < nd; d++) {
                    double dphi[4] = {0, 0, 0, 0};
                    for (int r = 0; r < 7; r++) {
                        if (r == 3)
                            continue;
                        long om = wrap_at(L, p, d, r - 3);
                        for (int a = 0; a < np; a++)
                            dphi[a] += D6[r] * prim[a * vol + om];
                    }
                    for (int jj = 0; jj < nd; jj++) {
                        double s = met[(d * nd + jj) * vol + o];
                        for (int a = 0; a < np; a++)
                            grad[a][jj] += s * dphi[a] / V;
                    }
                }
                double div = 0.0;
                for (int c = 0; c < nd; c++)
                    div += grad[c][c];
                double tau[3][3];
                for (int a = 0; a < nd; a++)
                    for (int b = 0; b < nd; b++)
                        tau[a][b] = mu * (grad[a][b] + grad[b][a] - (a == b ? 2.0 / 3.0 * div : 0.0));
                /* physical viscous fluxes Fv_jj, then contravariant ones */
                double F[3][NVMAX];
                for (int jj = 0; jj < nd; jj++) {
                    F[jj][0] = 0.0;
                    double work = 0.0;
                    for (int a = 0; a < nd; a++) {
                        F[jj][1 + a] = tau[a][jj];
                        work += prim[a * vol + o] * tau[a][jj];
                    }
                    F[jj][nv - 1] = work + kappa * grad[nd][jj];
                }
                for (int d = 0; d < nd; d++)
                    for (int v = 0; v < nv; v++) {
                        double sum = 0.0;
                        for (int jj = 0; jj < nd; jj++)
                            sum += met[(d * nd + jj) * vol + o] * F[jj][v];
                        fv[((long)d * nv + v) * vol + o] = sum;
                    }
            }
#pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < L->n[2]; k++)
        for (int j = 0; j < L->n[1]; j++)
            for (int i = 0; i < L->n[0]; i++) {
                int p[3] = {i, j, k};
                long o = at(L, i, j, k);
                for (int d = 0; d < nd; d++)
                    for (int r = 0; r < 7; r++) {
                        if (r == 3)
                            continue;
                        long om = wrap_at(L, p, d, r - 3);
                        for (int v = 0; v < nv; v++)
                            acc[v * vol + o] -= D6[r] * fv[((long)d * nv + v) * vol + om];
                    }
            }
    free(prim);
    free(fv);
    return 0;
}

/* residual of eq. (aderivative) summed over the directions in the order
 * xi, eta, zeta: dQ/dt = -(1/J)^{-1} sum_d (F'_{i+1/2} - F'_{i-1/2}) */
static int residual_filled(const layout *L, const fpo_scheme *sc, const double *met,
                           const double *qf, double *dqdt)
{
    long tot = (long)L->nv * L->vol;
    double *acc = (double *)calloc(tot, sizeof(double));
    if (!acc)
        return -1;
    for (int d = 0; d < L->ndim; d++) {
        int a, b;
        other_axes(d, &a, &b);
        int len = L->n[d] + 2 * L->g;
        int na = L->n[a], nb = L->n[b];
        double glf[3], *gp = NULL;
        if (sc->splitting) {
            glf_filled(L, sc, met, qf, d, glf);
            gp = glf;
        }
#pragma omp parallel
        {
            double *buf = (double *)malloc(sizeof(double) * len * (L->nv + 1 + L->ndim));
            double *F = (double *)malloc(sizeof(double) * (L->n[d] + 1) * NVMAX);
            line_t ln;
#pragma omp for collapse(2) schedule(static)
            for (int ib = 0; ib < nb; ib++)
                for (int ia = 0; ia < na; ia++) {
                    int p[3] = {0, 0, 0};
                    p[a] = ia;
                    p[b] = ib;
                    gather_line(L, qf, met, d, p, buf, &ln);
                    for (int f = 0; f <= L->n[d]; f++)
                        face_flux(sc, &ln, f - 1, gp, F + (long)f * NVMAX);
                    for (int i = 0; i < L->n[d]; i++) {
                        int c3[3] = {p[0], p[1], p[2]};
                        c3[d] = i;
                        long off = at(L, c3[0], c3[1], c3[2]);
                        for (int v = 0; v < L->nv; v++)
                            acc[v * L->vol + off] +=
                                F[(long)(i + 1) * NVMAX + v] - F[(long)i * NVMAX + v];
                    }
                }
            free(F);
            free(buf);
        }
    }
    if (sc->mu > 0.0 && viscous_acc(L, sc, met, qf, acc)) {
        free(acc);
        return -1;
    }
    memset(dqdt, 0, sizeof(double) * tot);
    for (int k = 0; k < L->n[2]; k++)
        for (int j = 0; j < L->n[1]; j++)
            for (int i = 0; i < L->n[0]; i++) {
                long off = at(L, i, j, k);
                double V = met[(L->nmet - 1) * L->vol + off];
                for (int v = 0; v < L->nv; v++)
                    dqdt[v * L->vol + off] = -acc[v * L->vol + off] / V;
            }
    free(acc);
    return 0;
}

int fpo_residual(const fpo_grid *gr, const fpo_scheme *sc, const double *met,
                 const double *q, double *dqdt)
{
    layout L;
    if (make_layout(gr, &L) || check_scheme(&L, sc) || !met || !q || !dqdt)
        return -1;
    double *qf = filled_copy(&L, q);
    if (!qf)
        return -1;
    int rc = residual_filled(&L, sc, met, qf, dqdt);
    free(qf);
    return rc;
}

/* (local speeds only: global ones need the whole block) */
int fpo_residual_at(const fpo_grid *gr, const fpo_scheme *sc, const double *met,
                    const double *q, int npts, const int *ijk, double *out)
{
    layout L;
    if (make_layout(gr, &L) || check_scheme(&L, sc) || npts < 0 || sc->splitting || sc->mu > 0.0)
        return -1;
    for (int t = 0; t < npts; t++)
        for (int d = 0; d < L.ndim; d++) {
            int c = ijk[3 * t + d];
            if (c < 0 || c >= L.n[d])
                return -1;
        }
    int maxlen = 0;
    for (int d = 0; d < L.ndim; d++)
        if (L.n[d] + 2 * L.g > maxlen)
            maxlen = L.n[d] + 2 * L.g;
#pragma omp parallel
    {
        double *buf = (double *)malloc(sizeof(double) * maxlen * (L.nv + 1 + L.ndim));
        double *qline = (double *)malloc(sizeof(double) * maxlen * L.nv);
        line_t ln;
#pragma omp for schedule(dynamic, 8)
        for (int t = 0; t < npts; t++) {
            int p[3] = {ijk[3 * t], ijk[3 * t + 1], L.ndim == 3 ? ijk[3 * t + 2] : 0};
            double acc[NVMAX] = {0, 0, 0, 0, 0};
            for (int d = 0; d < L.ndim; d++) {
                gather_line(&L, q, met, d, p, buf, &ln);
                /* periodic ghost values come from the periodic image */
                int len = L.n[d] + 2 * L.g;
                if (L.bc[d] == 0) {
                    for (int v = 0; v < L.nv; v++) {
                        for (int tt = 0; tt < len; tt++) {
                            int node = tt - L.g;
                            int src = ((node % L.n[d]) + L.n[d]) % L.n[d];
                            qline[v * len + tt] = ln.Q[v][src];
                        }
                        memcpy(buf + v * len, qline + v * len, sizeof(double) * len);
                    }
                }
                double Fm[NVMAX], Fpl[NVMAX];
                face_flux(sc, &ln, p[d] - 1, NULL, Fm);
                face_flux(sc, &ln, p[d], NULL, Fpl);
                for (int v = 0; v < L.nv; v++)
                    acc[v] += Fpl[v] - Fm[v];
            }
            double V = met[(L.nmet - 1) * L.vol + at(&L, p[0], p[1], p[2])];
            for (int v = 0; v < L.nv; v++)
                out[(long)L.nv * t + v] = -acc[v] / V;
        }
        free(qline);
        free(buf);
    }
    return 0;
}

/* The residual at selected interior nodes with the metrics evaluated on the
 * fly from the coordinates (no metric array): for each direction the line
 * through the node is gathered over the reach of its two faces only. */
int fpo_residual_at_xyz(const fpo_grid *gr, const fpo_scheme *sc, const double *xyz,
                        const double *q, int npts, const int *ijk, double *out)
{
    layout L;
    cgrid C;
    if (make_layout(gr, &L) || check_scheme(&L, sc) || sc->splitting || sc->mu > 0.0 ||
        make_cgrid(&L, sc->Y, xyz, &C) || npts < 0)
        return -1;
    for (int t = 0; t < npts; t++)
        for (int d = 0; d < L.ndim; d++) {
            int c = ijk[3 * t + d];
            if (c < 0 || c >= L.n[d])
                return -1;
        }
    /* reach of the two faces of a node: the 6-point stencil (3 nodes) and
     * the face interpolation (Y/2 nodes); the ghost width covers both */
    const int R = L.g;
    const int len = 2 * R + 1;
#pragma omp parallel for schedule(dynamic, 4)
    for (int t = 0; t < npts; t++) {
        int p[3] = {ijk[3 * t], ijk[3 * t + 1], L.ndim == 3 ? ijk[3 * t + 2] : 0};
        double buf[(NVMAX + 1 + 3) * 17];
        double acc[NVMAX] = {0, 0, 0, 0, 0};
        double Vp = 0.0;
        for (int d = 0; d < L.ndim; d++) {
            int nsd = L.ndim;
            for (int m = -R; m <= R; m++) {
                int c3[3] = {p[0], p[1], p[2]};
                c3[d] = p[d] + m;
                /* state: periodic image or frozen ghost value */
                int s3[3] = {c3[0], c3[1], c3[2]};
                if (L.bc[d] == 0)
                    s3[d] = ((c3[d] % L.n[d]) + L.n[d]) % L.n[d];
                long off = at(&L, s3[0], s3[1], s3[2]);
                for (int v = 0; v < L.nv; v++)
                    buf[v * len + m + R] = q[v * L.vol + off];
                double mt[10];
                metrics_node(&C, c3, mt);
                buf[L.nv * len + m + R] = mt[L.nmet - 1];
                for (int c = 0; c < nsd; c++)
                    buf[(L.nv + 1 + c) * len + m + R] = mt[d * nsd + c];
                if (m == 0)
                    Vp = mt[L.nmet - 1];
            }
            line_t ln;
            ln.ndim = L.ndim;
            ln.nv = L.nv;
            for (int v = 0; v < L.nv; v++)
                ln.Q[v] = buf + v * len + R - p[d];
            ln.V = buf + L.nv * len + R - p[d];
            for (int c = 0; c < nsd; c++)
                ln.S[c] = buf + (L.nv + 1 + c) * len + R - p[d];
            double Fm[NVMAX], Fpl[NVMAX];
            face_flux(sc, &ln, p[d] - 1, NULL, Fm);
            face_flux(sc, &ln, p[d], NULL, Fpl);
            for (int v = 0; v < L.nv; v++)
                acc[v] += Fpl[v] - Fm[v];
        }
        for (int v = 0; v < L.nv; v++)
            out[(long)L.nv * t + v] = -acc[v] / Vp;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* boundary faces (the wall-bounded cases of Sec. 4)                        */
/* ------------------------------------------------------------------------ */

static int check_bcs(const layout *L, const fpo_bcs *bcs)
{
    for (int a = 0; a < L->ndim; a++)
        for (int sd = 0; sd < 2; sd++) {
            int k = bcs->kind[a][sd];
            if (k < 0 || k > 3)
                return -1;
            if (k && L->bc[a] == 0)
                return -1; /* periodic axes have no boundary faces */
            if (k == 2 && L->n[a] < L->g + 1)
                return -1; /* the mirror images must be interior nodes */
            if (k == 3 && !bcs->nodes)
                return -1;
        }
    return 0;
}

/* fill the ghost layers of the boundary faces at time t */
static void apply_bcs_layout(const layout *L, const fpo_bcs *bcs, const double *met, double *q, double t)
{
    const int nv = L->nv, ndim = L->ndim;
    for (int a = 0; a < ndim; a++) {
        if (L->bc[a] == 0)
            continue;
        int e1, e2;
        other_axes(a, &e1, &e2);
        int n1 = L->n[e1], n2 = e2 < ndim ? L->n[e2] : 1;
        for (int sd = 0; sd < 2; sd++) {
            int kind = bcs->kind[a][sd];
            if (kind == 0)
                continue;
            int bnode = sd ? L->n[a] - 1 : 0; /* the boundary node along axis a */
            for (int i2 = 0; i2 < n2; i2++)
                for (int i1 = 0; i1 < n1; i1++) {
                    if (bcs->mask[a][sd] && !bcs->mask[a][sd][(long)i2 * n1 + i1])
                        continue;
                    int p[3] = {0, 0, 0};
                    p[e1] = i1;
                    if (e2 < ndim)
                        p[e2] = i2;
                    /* wall normal: the metric vector of axis a at the boundary node */
                    double nw[3] = {0, 0, 0};
                    if (kind == 2) {
                        p[a] = bnode;
                        long ob = at(L, p[0], p[1], p[2]);
                        double nn = 0.0;
                        for (int c = 0; c < ndim; c++) {
                            nw[c] = met[(a * ndim + c) * L->vol + ob];
                            nn += nw[c] * nw[c];
                        }
                        nn = sqrt(nn);
                        for (int c = 0; c < ndim; c++)
                            nw[c] /= nn;
                    }
                    for (int l = 1; l <= L->g; l++) {
                        p[a] = sd ? L->n[a] - 1 + l : -l;
                        long og = at(L, p[0], p[1], p[2]);
                        double Q[NVMAX];
                        if (kind == 1) { /* zeroth-order extrapolation */
                            p[a] = bnode;
                            long os = at(L, p[0], p[1], p[2]);
                            for (int v = 0; v < nv; v++)
                                Q[v] = q[v * L->vol + os];
                        } else if (kind == 2) { /* mirror image, normal velocity reversed */
                            p[a] = sd ? L->n[a] - 1 - l : l;
                            long os = at(L, p[0], p[1], p[2]);
                            double un = 0.0;
                            for (int c = 0; c < ndim; c++)
                                un += nw[c] * q[(1 + c) * L->vol + os];
                            Q[0] = q[os];
                            for (int c = 0; c < ndim; c++)
                                Q[1 + c] = q[(1 + c) * L->vol + os] - 2.0 * un * nw[c];
                            Q[nv - 1] = q[(nv - 1) * L->vol + os];
                        } else { /* moving planar shock */
                            double xn = 0.0;
                            for (int c = 0; c < ndim; c++)
                                xn += bcs->normal[c] * bcs->nodes[c * L->vol + og];
                            const double *src = xn < bcs->offset + bcs->speed * t ? bcs->post : bcs->pre;
                            for (int v = 0; v < nv; v++)
                                Q[v] = src[v];
                        }
                        for (int v = 0; v < nv; v++)
                            q[v * L->vol + og] = Q[v];
                    }
                }
        }
    }
}

int fpo_apply_bcs(const fpo_grid *gr, const fpo_bcs *bcs, const double *met, double *q, double t)
{
    layout L;
    if (make_layout(gr, &L) || !bcs || !met || !q || check_bcs(&L, bcs))
        return -1;
    apply_bcs_layout(&L, bcs, met, q, t);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* third-order TVD Runge-Kutta (Sec. 2.2)                                   */
/* ------------------------------------------------------------------------ */

/* Q1 = Qn + dt L(Qn); Q2 = 3/4 Qn + 1/4 (Q1 + dt L(Q1));
 * Qn+1 = 1/3 Qn + 2/3 (Q2 + dt L(Q2)); interior nodes only.  With boundary
 * faces, each stage's input gets its ghost layers at the stage's time
 * t, t + dt, t + dt/2. */
static int rk3_step_layout(const layout *L, const fpo_scheme *sc, const fpo_bcs *bcs,
                           const double *met, double *q, double t, double dt)
{
    long tot = (long)L->nv * L->vol;
    double *q0 = (double *)malloc(sizeof(double) * tot);
    double *qs = (double *)malloc(sizeof(double) * tot);
    double *k = (double *)malloc(sizeof(double) * tot);
    if (!q0 || !qs || !k) {
        free(q0);
        free(qs);
        free(k);
        return -1;
    }
    memcpy(q0, q, sizeof(double) * tot);
    memcpy(qs, q, sizeof(double) * tot);
    const double a[3] = {0.0, 3.0 / 4.0, 1.0 / 3.0};
    const double b[3] = {1.0, 1.0 / 4.0, 2.0 / 3.0};
    const double c[3] = {0.0, 1.0, 0.5};
    int rc = 0;
    for (int st = 0; st < 3 && !rc; st++) {
        if (bcs)
            apply_bcs_layout(L, bcs, met, qs, t + c[st] * dt);
        double *qf = filled_copy(L, qs);
        if (!qf) {
            rc = -1;
            break;
        }
        rc = residual_filled(L, sc, met, qf, k);
        free(qf);
        for (int v = 0; v < L->nv; v++)
            for (int kk = 0; kk < L->n[2]; kk++)
                for (int j = 0; j < L->n[1]; j++)
                    for (int i = 0; i < L->n[0]; i++) {
                        long off = v * L->vol + at(L, i, j, kk);
                        double upd = qs[off] + dt * k[off];
                        qs[off] = st == 0 ? upd : a[st] * q0[off] + b[st] * upd;
                    }
    }
    if (!rc)
        memcpy(q, qs, sizeof(double) * tot);
    free(q0);
    free(qs);
    free(k);
    return rc;
}

int fpo_rk3_step(const fpo_grid *gr, const fpo_scheme *sc, const double *met,
                 double *q, double dt)
{
    layout L;
    if (make_layout(gr, &L) || check_scheme(&L, sc) || !met || !q)
        return -1;
    return rk3_step_layout(&L, sc, NULL, met, q, 0.0, dt);
}

int fpo_solve(const fpo_grid *gr, const fpo_scheme *sc, const double *met, double *q,
              double dt, long nsteps)
{
    for (long s = 0; s < nsteps; s++) {
        int rc = fpo_rk3_step(gr, sc, met, q, dt);
        if (rc)
            return rc;
    }
    return 0;
}

int fpo_solve_bcs(const fpo_grid *gr, const fpo_scheme *sc, const fpo_bcs *bcs, const double *met,
                  double *q, double t0, double dt, long nsteps)
{
    layout L;
    if (make_layout(gr, &L) || check_scheme(&L, sc) || !bcs || !met || !q || check_bcs(&L, bcs))
        return -1;
    for (long s = 0; s < nsteps; s++) {
        int rc = rk3_step_layout(&L, sc, bcs, met, q, t0 + s * dt, dt);
        if (rc)
            return rc;
    }
    return 0;
}

double fpo_max_dt(const fpo_grid *gr, const fpo_scheme *sc, const double *met,
                  const double *q, double cfl)
{
    layout L;
    if (make_layout(gr, &L) || !sc)
        return -1.0;
    double mx = 0.0;
    for (int k = 0; k < L.n[2]; k++)
        for (int j = 0; j < L.n[1]; j++)
            for (int i = 0; i < L.n[0]; i++) {
                long off = at(&L, i, j, k);
                double Q[NVMAX];
                for (int v = 0; v < L.nv; v++)
                    Q[v] = q[v * L.vol + off];
                double c = sqrt(sc->gamma * pressure(L.ndim, sc->gamma, Q) / Q[0]);
                double V = met[(L.nmet - 1) * L.vol + off];
                double sum = 0.0;
                for (int d = 0; d < L.ndim; d++) {
                    double su = 0.0, s2 = 0.0;
                    for (int c2 = 0; c2 < L.ndim; c2++) {
                        double s = met[(d * L.ndim + c2) * L.vol + off];
                        su += s * Q[1 + c2] / Q[0];
                        s2 += s * s;
                    }
                    sum += fabs(su) + c * sqrt(s2);
                }
                sum /= V;
                if (sum > mx)
                    mx = sum;
            }
    return cfl / mx;
}

int fpo_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void fpo_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}
