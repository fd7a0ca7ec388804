/*
 * numa_oracle.c -- plain, slow, FP64 CPU oracle for the NUMA spectral-element
 * right-hand side, direct stiffness summation and SSP-RK3 step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  The product path
 * (the HIP library) shares no code, header, table or helper with it.
 *
 * Every routine follows the paper (Mueller et al., "Strong scaling for
 * numerical weather prediction at petascale with the atmospheric model NUMA",
 * IJHPCA 2016) section by section:
 *   - Lagrange basis on Lobatto points:        Sec. "Spatial Discretization", Eq. (expansion)
 *   - strong form with diagonal mass matrix:   Eq. (discstrongform)
 *   - derivative contractions + chain rule:    Eq. (derivatives) (garbled index/metric
 *                                              read as the standard chain rule)
 *   - DSS weighted by element volume, M^-1:    text after Eq. (derivatives); Code example 1
 *   - explicit RK stage update ("update q"):   Sec. "Time Discretization"; Code example 1
 * Readings where the paper is silent (variable set, EOS form, reference
 * atmosphere, no-flux projection, SSP-RK3, mesh numbering) are listed in the
 * design notes of the repository; each is restated at the routine using it.
 *
 * Loops are plain and in the paper's order.  Build: gcc -O2 -ffp-contract=off
 * (no FMA contraction), optional -fopenmp (parallel over elements or over
 * unique nodes only; results do not depend on the thread count).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXP 9 /* N <= 8 */

typedef struct {
    int32_t kind;        /* 0 = box, 1 = cubed-sphere shell */
    int32_t N;           /* polynomial order p of the paper */
    int32_t ne[3];       /* box: nx, ny, nz; shell: ne (per cube edge), unused, nz */
    int32_t periodic[3]; /* box only: x and y must be periodic; z either */
    double extent[3];    /* box: Lx, Ly, H; shell: a (radius), unused, H */
    double h0;           /* box terrain amplitude */
} or_mesh_desc;

typedef struct {
    double R, cp, g0, p0;
    double T0; /* box: theta0 of the isentropic reference; shell: isothermal T */
} or_phys;

typedef struct {
    int32_t kind;     /* 0 rest, 1 cosine bubble (box), 2 zonal jet + gaussian blob (shell) */
    double amp;       /* bubble / blob amplitude [K] */
    double radius;    /* bubble radius [m]; blob horizontal e-folding length [m] */
    double c[3];      /* bubble centre x,y,z [m]; blob lon, lat [rad], height [m] */
    double lz;        /* blob vertical e-folding length [m] */
    double jet_u0;    /* jet speed [m/s] */
    double noise_amp; /* scale applied to the standard-normal noise on u, v, w */
} or_ic_desc;

typedef struct {
    or_mesh_desc m;
    or_phys ph;
    int N, P, np;
    int64_t ne, nl, nu, nh, nk;
    double xi[OR_MAXP], w[OR_MAXP], D[OR_MAXP * OR_MAXP];
    int32_t *G;      /* [ne][np] gather map: element-local -> unique */
    double *xl;      /* [3][nl] element-local coordinates */
    double *xu;      /* [3][nu] unique-node coordinates */
    double *dl, *hl; /* shell: [3][nl] unit radial direction, [nl] height above the inner radius */
    double *du, *hu; /* shell: the same at unique nodes */
    double *met;     /* [10][nl] xi_x xi_y xi_z eta_x eta_y eta_z zeta_x zeta_y zeta_z J*w */
    double *M;       /* [nu] diagonal mass matrix */
    double *ref;     /* [3][nu] rho_bar, theta_bar, p_bar */
    double *grav;    /* [3][nu] gravity vector */
    double *nrm;     /* [3][nu] outward unit normal at no-flux nodes, 0 elsewhere */
    int32_t *isbnd;  /* [nu] 1 at no-flux boundary nodes */
    int64_t *off;    /* [nu+1] inverse map offsets */
    int64_t *cp;     /* [nl] copies of each unique node, ascending e*np+l */
    int dtheta;      /* theta_bar varies in space (shell): its gradient enters R_theta */
} or_ctx;

static const double OR_PI = 3.14159265358979323846;

/* ------------------------------------------------------------------------ */
/* Legendre polynomial P_n(x) and derivative by the three-term recurrence.   */
static void legendre(int n, double x, double *Pn, double *dPn, double *Pn1)
{
    double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
    if (n == 0) { *Pn = 1.0; *dPn = 0.0; *Pn1 = 0.0; return; }
    for (int k = 1; k < n; k++) {
        double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
        double d2 = d0 + (2.0 * k + 1.0) * p1;
        p0 = p1; p1 = p2; d0 = d1; d1 = d2;
    }
    *Pn = p1; *dPn = d1; *Pn1 = p0;
}

/*
 * GLL nodes, weights and derivative matrix (Sec. "Spatial Discretization":
 * Lobatto points, Lagrange basis psi_i, derivative dpsi_m/dxi at xi_i).
 * Nodes: -1, +1 and the roots of q(x) = P_{N-1}(x) - x P_N(x) (proportional to
 * (1-x^2) P_N'(x)), by Newton from the Chebyshev-Lobatto points.
 * Weights: w_i = 2 / (N (N+1) P_N(x_i)^2).
 * D_im = dpsi_m/dxi (xi_i) = P_N(x_i) / (P_N(x_m) (x_i - x_m)), i != m;
 * D_00 = -N(N+1)/4, D_NN = N(N+1)/4, other diagonal entries 0.
 * D is row-major: D[i*(N+1)+m].
 */
int or_gll(int N, double *xi, double *w, double *D)
{
    if (N < 1 || N > 8) return -1;
    int P = N + 1;
    for (int i = 0; i <= N; i++) xi[i] = -cos(OR_PI * i / N);
    for (int i = 1; i < N; i++) {
        double x = xi[i];
        for (int it = 0; it < 100; it++) {
            double pn, dpn, pn1, pm, dpm, pm1;
            legendre(N, x, &pn, &dpn, &pn1);
            legendre(N - 1, x, &pm, &dpm, &pm1);
            double q = pm - x * pn;
            double dq = dpm - pn - x * dpn;
            double dx = q / dq;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        xi[i] = x;
    }
    xi[0] = -1.0; xi[N] = 1.0;
    for (int i = 0; i < P / 2; i++) { double s = 0.5 * (xi[N - i] - xi[i]); xi[i] = -s; xi[N - i] = s; }
    if (N % 2 == 0) xi[N / 2] = 0.0;
    double PN[OR_MAXP];
    for (int i = 0; i <= N; i++) {
        double pn, dpn, pn1;
        legendre(N, xi[i], &pn, &dpn, &pn1);
        PN[i] = pn;
        w[i] = 2.0 / (N * (N + 1.0) * pn * pn);
    }
    for (int i = 0; i <= N; i++)
        for (int m = 0; m <= N; m++) {
            double d;
            if (i != m) d = PN[i] / (PN[m] * (xi[i] - xi[m]));
            else if (i == 0) d = -N * (N + 1.0) / 4.0;
            else if (i == N) d = N * (N + 1.0) / 4.0;
            else d = 0.0;
            D[i * P + m] = d;
        }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Mesh numbering.  Local node l = i + P(j + P k); unique ids follow a global
 * lattice (CG storage: one copy per unique grid point).
 *
 * Box: e = ex + nx(ey + ny ez); lattice g = (ex N + i, ey N + j, ez N + k),
 * wrapped in periodic directions; id = gi + ni (gj + nj gk).
 *
 * Shell: a cube surface lattice (X,Y,Z) in {0..L}^3, L = ne N.  Face f maps
 * (s,t) in {0..L}^2 to: f0 (L,s,t), f1 (L-s,L,t), f2 (0,L-s,t), f3 (s,0,t),
 * f4 (s,t,L), f5 (t,s,0).  Horizontal ids are given in first-occurrence order
 * over f, then t, then s; id = h + nh gk.  e = ex + ne(ey + ne(f + 6 ez)).
 */
static void face_lattice(int f, int L, int s, int t, int *X, int *Y, int *Z)
{
    switch (f) {
    case 0: *X = L; *Y = s; *Z = t; break;
    case 1: *X = L - s; *Y = L; *Z = t; break;
    case 2: *X = 0; *Y = L - s; *Z = t; break;
    case 3: *X = s; *Y = 0; *Z = t; break;
    case 4: *X = s; *Y = t; *Z = L; break;
    default: *X = t; *Y = s; *Z = 0; break;
    }
}

static int check_desc(const or_mesh_desc *d)
{
    if (d->N < 1 || d->N > 8) return -1;
    if (d->kind == 0) {
        for (int a = 0; a < 3; a++) if (d->ne[a] < 1) return -1;
        if (!d->periodic[0] || !d->periodic[1]) return -1;
        for (int a = 0; a < 3; a++) if (d->periodic[a] && d->ne[a] < 2) return -1;
        return 0;
    }
    if (d->kind == 1) return (d->ne[0] >= 1 && d->ne[2] >= 1) ? 0 : -1;
    return -1;
}

/* coordinate of lattice index c in [0, ncell*N] along one direction:
 * the element (clamped to the last) and its local node */
static void lattice_split(int64_t c, int N, int ncell, int *ec, int *ic)
{
    int64_t e = c / N;
    if (e > ncell - 1) e = ncell - 1;
    *ec = (int)e;
    *ic = (int)(c - (int64_t)N * e);
}

static void box_point(const or_ctx *C, int64_t gi, int64_t gj, int64_t gk, double *x, double *y, double *z)
{
    const or_mesh_desc *d = &C->m;
    int N = C->N, e, i;
    lattice_split(gi, N, d->ne[0], &e, &i);
    double xx = d->extent[0] * (e + (1.0 + C->xi[i]) / 2.0) / d->ne[0];
    lattice_split(gj, N, d->ne[1], &e, &i);
    double yy = d->extent[1] * (e + (1.0 + C->xi[i]) / 2.0) / d->ne[1];
    lattice_split(gk, N, d->ne[2], &e, &i);
    double zz = d->extent[2] * (e + (1.0 + C->xi[i]) / 2.0) / d->ne[2];
    /* terrain-following map z' = z + h(x,y) (1 - z/H) */
    double h = d->h0 * sin(2.0 * OR_PI * xx / d->extent[0]) * sin(2.0 * OR_PI * yy / d->extent[1]);
    *x = xx; *y = yy; *z = zz + h * (1.0 - zz / d->extent[2]);
}

/* equiangular gnomonic node from the surface lattice (X,Y,Z) and radial
 * lattice index gk: unit direction dir = P/|P| with P = (tan alpha(X),
 * tan alpha(Y), tan alpha(Z)), height hgt above the inner radius a, and the
 * position (a + hgt) dir. */
static void shell_point(const or_ctx *C, int X, int Y, int Z, int64_t gk, double *dir, double *hgt, double *pos)
{
    const or_mesh_desc *d = &C->m;
    int N = C->N, ne = d->ne[0], e, i;
    int lat[3] = {X, Y, Z};
    double Pv[3];
    for (int a = 0; a < 3; a++) {
        lattice_split(lat[a], N, ne, &e, &i);
        double alpha = (OR_PI / 2.0) * (e + (1.0 + C->xi[i]) / 2.0) / ne - OR_PI / 4.0;
        Pv[a] = tan(alpha);
    }
    double nrm = sqrt(Pv[0] * Pv[0] + Pv[1] * Pv[1] + Pv[2] * Pv[2]);
    lattice_split(gk, N, d->ne[2], &e, &i);
    double h = d->extent[2] * (e + (1.0 + C->xi[i]) / 2.0) / d->ne[2];
    double r = d->extent[0] + h;
    for (int a = 0; a < 3; a++) {
        dir[a] = Pv[a] / nrm;
        pos[a] = r * dir[a];
    }
    *hgt = h;
}

int or_counts(const or_mesh_desc *d, int64_t *n_elem, int64_t *n_unique, int64_t *n_horiz)
{
    if (check_desc(d)) return -1;
    int N = d->N;
    if (d->kind == 0) {
        int64_t ni = d->periodic[0] ? (int64_t)d->ne[0] * N : (int64_t)d->ne[0] * N + 1;
        int64_t nj = d->periodic[1] ? (int64_t)d->ne[1] * N : (int64_t)d->ne[1] * N + 1;
        int64_t nk = d->periodic[2] ? (int64_t)d->ne[2] * N : (int64_t)d->ne[2] * N + 1;
        *n_elem = (int64_t)d->ne[0] * d->ne[1] * d->ne[2];
        *n_horiz = ni * nj;
        *n_unique = ni * nj * nk;
    } else {
        int64_t L = (int64_t)d->ne[0] * N;
        *n_elem = 6 * (int64_t)d->ne[0] * d->ne[0] * d->ne[2];
        *n_horiz = 6 * L * L + 2;
        *n_unique = *n_horiz * ((int64_t)d->ne[2] * N + 1);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
static void build_numbering(or_ctx *C)
{
    const or_mesh_desc *d = &C->m;
    int N = C->N, P = C->P, np = C->np;
    if (d->kind == 0) {
        int nx = d->ne[0], ny = d->ne[1], nz = d->ne[2];
        int64_t ni = d->periodic[0] ? (int64_t)nx * N : (int64_t)nx * N + 1;
        int64_t nj = d->periodic[1] ? (int64_t)ny * N : (int64_t)ny * N + 1;
        int64_t nk = d->periodic[2] ? (int64_t)nz * N : (int64_t)nz * N + 1;
        for (int ez = 0; ez < nz; ez++)
            for (int ey = 0; ey < ny; ey++)
                for (int ex = 0; ex < nx; ex++) {
                    int64_t e = ex + (int64_t)nx * (ey + (int64_t)ny * ez);
                    for (int k = 0; k < P; k++)
                        for (int j = 0; j < P; j++)
                            for (int i = 0; i < P; i++) {
                                int64_t gi = (int64_t)ex * N + i, gj = (int64_t)ey * N + j, gk = (int64_t)ez * N + k;
                                if (d->periodic[0]) gi %= ni;
                                if (d->periodic[1]) gj %= nj;
                                if (d->periodic[2]) gk %= nk;
                                C->G[e * np + i + P * (j + P * k)] = (int32_t)(gi + ni * (gj + nj * gk));
                            }
                }
        C->nk = nk;
    } else {
        int ne = d->ne[0], nz = d->ne[2];
        int L = ne * N;
        int64_t L1 = L + 1;
        int32_t *hid = (int32_t *)malloc(sizeof(int32_t) * L1 * L1 * L1);
        for (int64_t a = 0; a < L1 * L1 * L1; a++) hid[a] = -1;
        int32_t next = 0;
        for (int f = 0; f < 6; f++)
            for (int t = 0; t <= L; t++)
                for (int s = 0; s <= L; s++) {
                    int X, Y, Z;
                    face_lattice(f, L, s, t, &X, &Y, &Z);
                    int64_t a = X + L1 * (Y + L1 * Z);
                    if (hid[a] < 0) hid[a] = next++;
                }
        int64_t nh = C->nh;
        for (int ez = 0; ez < nz; ez++)
            for (int f = 0; f < 6; f++)
                for (int ey = 0; ey < ne; ey++)
                    for (int ex = 0; ex < ne; ex++) {
                        int64_t e = ex + (int64_t)ne * (ey + (int64_t)ne * (f + 6 * (int64_t)ez));
                        for (int k = 0; k < P; k++)
                            for (int j = 0; j < P; j++)
                                for (int i = 0; i < P; i++) {
                                    int X, Y, Z;
                                    face_lattice(f, L, ex * N + i, ey * N + j, &X, &Y, &Z);
                                    int64_t h = hid[X + L1 * (Y + L1 * Z)];
                                    int64_t gk = (int64_t)ez * N + k;
                                    C->G[e * np + i + P * (j + P * k)] = (int32_t)(h + nh * gk);
                                }
                    }
        /* unique coordinates: any lattice point (the first occurrence) */
        for (int f = 0; f < 6; f++)
            for (int t = 0; t <= L; t++)
                for (int s = 0; s <= L; s++) {
                    int X, Y, Z;
                    face_lattice(f, L, s, t, &X, &Y, &Z);
                    int64_t h = hid[X + L1 * (Y + L1 * Z)];
                    for (int64_t gk = 0; gk < C->nk; gk++) {
                        double dir[3], hgt, pos[3];
                        shell_point(C, X, Y, Z, gk, dir, &hgt, pos);
                        int64_t I = h + nh * gk;
                        for (int a = 0; a < 3; a++) {
                            C->xu[a * C->nu + I] = pos[a];
                            C->du[a * C->nu + I] = dir[a];
                        }
                        C->hu[I] = hgt;
                    }
                }
        /* element-local coordinates from the same lattice: copies agree bitwise */
        for (int ez = 0; ez < nz; ez++)
            for (int f = 0; f < 6; f++)
                for (int ey = 0; ey < ne; ey++)
                    for (int ex = 0; ex < ne; ex++) {
                        int64_t e = ex + (int64_t)ne * (ey + (int64_t)ne * (f + 6 * (int64_t)ez));
                        for (int k = 0; k < P; k++)
                            for (int j = 0; j < P; j++)
                                for (int i = 0; i < P; i++) {
                                    int X, Y, Z;
                                    face_lattice(f, L, ex * N + i, ey * N + j, &X, &Y, &Z);
                                    double dir[3], hgt, pos[3];
                                    shell_point(C, X, Y, Z, (int64_t)ez * N + k, dir, &hgt, pos);
                                    int64_t g = e * np + i + P * (j + P * k);
                                    for (int a = 0; a < 3; a++) {
                                        C->xl[a * C->nl + g] = pos[a];
                                        C->dl[a * C->nl + g] = dir[a];
                                    }
                                    C->hl[g] = hgt;
                                }
                    }
        free(hid);
    }
    if (d->kind == 0) {
        /* element-local coordinates (unwrapped) and unique coordinates (wrapped lattice) */
        int nx = d->ne[0], ny = d->ne[1], nz = d->ne[2];
        for (int ez = 0; ez < nz; ez++)
            for (int ey = 0; ey < ny; ey++)
                for (int ex = 0; ex < nx; ex++) {
                    int64_t e = ex + (int64_t)nx * (ey + (int64_t)ny * ez);
                    for (int k = 0; k < P; k++)
                        for (int j = 0; j < P; j++)
                            for (int i = 0; i < P; i++) {
                                double x, y, z;
                                box_point(C, (int64_t)ex * N + i, (int64_t)ey * N + j, (int64_t)ez * N + k, &x, &y, &z);
                                int64_t g = e * np + i + P * (j + P * k);
                                C->xl[g] = x; C->xl[C->nl + g] = y; C->xl[2 * C->nl + g] = z;
                            }
                }
        int64_t ni = d->periodic[0] ? (int64_t)nx * N : (int64_t)nx * N + 1;
        int64_t nj = d->periodic[1] ? (int64_t)ny * N : (int64_t)ny * N + 1;
        for (int64_t gk = 0; gk < C->nk; gk++)
            for (int64_t gj = 0; gj < nj; gj++)
                for (int64_t gi = 0; gi < ni; gi++) {
                    double x, y, z;
                    box_point(C, gi, gj, gk, &x, &y, &z);
                    int64_t I = gi + ni * (gj + nj * gk);
                    C->xu[I] = x; C->xu[C->nu + I] = y; C->xu[2 * C->nu + I] = z;
                }
    }
}

/* Inverse map: copies of each unique node in ascending (e*np + l). */
static void build_inverse(or_ctx *C)
{
    int64_t *cnt = (int64_t *)calloc(C->nu + 1, sizeof(int64_t));
    for (int64_t g = 0; g < C->nl; g++) cnt[C->G[g] + 1]++;
    C->off[0] = 0;
    for (int64_t I = 0; I < C->nu; I++) C->off[I + 1] = C->off[I] + cnt[I + 1];
    int64_t *fill = (int64_t *)calloc(C->nu, sizeof(int64_t));
    for (int64_t g = 0; g < C->nl; g++) {
        int64_t I = C->G[g];
        C->cp[C->off[I] + fill[I]++] = g;
    }
    free(cnt); free(fill);
}

/*
 * Metric terms (computed once, Eq. (derivatives) and the remark after it):
 * A = d(x,y,z)/d(xi,eta,zeta) by derivative-matrix contractions of the nodal
 * coordinates (isoparametric), J = det A, inverse metric = adj(A)/J.
 * Stored with J w_i w_j w_k (the weight of Eq. (discstrongform)).
 * On the shell the nodal coordinates are x = (a + h_k) d_ij, so the same sums
 * are taken factor by factor: d/dxi and d/deta contract the unit directions
 * (the radius is constant along them), d/dzeta contracts the heights h (the
 * direction is constant along it, and the contraction annihilates the constant
 * radius a).  This avoids rounding the coordinates at the planet's radius
 * before differencing them over elements a few km deep.
 */
static int build_metric(or_ctx *C)
{
    int P = C->P, np = C->np;
    int bad = 0;
#pragma omp parallel for reduction(| : bad)
    for (int64_t e = 0; e < C->ne; e++) {
        const double *X = C->xl + e * np, *Y = C->xl + C->nl + e * np, *Z = C->xl + 2 * C->nl + e * np;
        for (int k = 0; k < P; k++)
            for (int j = 0; j < P; j++)
                for (int i = 0; i < P; i++) {
                    int l = i + P * (j + P * k);
                    double xa = 0, xb = 0, xc = 0, ya = 0, yb = 0, yc = 0, za = 0, zb = 0, zc = 0;
                    if (C->m.kind == 0) {
                        for (int m = 0; m < P; m++) {
                            int la = m + P * (j + P * k), lb = i + P * (m + P * k), lc = i + P * (j + P * m);
                            xa += C->D[i * P + m] * X[la]; ya += C->D[i * P + m] * Y[la]; za += C->D[i * P + m] * Z[la];
                            xb += C->D[j * P + m] * X[lb]; yb += C->D[j * P + m] * Y[lb]; zb += C->D[j * P + m] * Z[lb];
                            xc += C->D[k * P + m] * X[lc]; yc += C->D[k * P + m] * Y[lc]; zc += C->D[k * P + m] * Z[lc];
                        }
                    } else {
                        const double *DX = C->dl + e * np, *DY = C->dl + C->nl + e * np, *DZ = C->dl + 2 * C->nl + e * np;
                        const double *Hh = C->hl + e * np;
                        double r = C->m.extent[0] + Hh[l], hz = 0.0;
                        for (int m = 0; m < P; m++) {
                            int la = m + P * (j + P * k), lb = i + P * (m + P * k), lc = i + P * (j + P * m);
                            xa += C->D[i * P + m] * DX[la]; ya += C->D[i * P + m] * DY[la]; za += C->D[i * P + m] * DZ[la];
                            xb += C->D[j * P + m] * DX[lb]; yb += C->D[j * P + m] * DY[lb]; zb += C->D[j * P + m] * DZ[lb];
                            hz += C->D[k * P + m] * Hh[lc];
                        }
                        xa *= r; ya *= r; za *= r; xb *= r; yb *= r; zb *= r;
                        xc = hz * DX[l]; yc = hz * DY[l]; zc = hz * DZ[l];
                    }
                    double J = xa * (yb * zc - yc * zb) - xb * (ya * zc - yc * za) + xc * (ya * zb - yb * za);
                    if (!(J > 0.0)) bad = 1;
                    double inv[9];
                    inv[0] = (yb * zc - yc * zb) / J; /* xi_x   */
                    inv[1] = (xc * zb - xb * zc) / J; /* xi_y   */
                    inv[2] = (xb * yc - xc * yb) / J; /* xi_z   */
                    inv[3] = (yc * za - ya * zc) / J; /* eta_x  */
                    inv[4] = (xa * zc - xc * za) / J; /* eta_y  */
                    inv[5] = (xc * ya - xa * yc) / J; /* eta_z  */
                    inv[6] = (ya * zb - yb * za) / J; /* zeta_x */
                    inv[7] = (xb * za - xa * zb) / J; /* zeta_y */
                    inv[8] = (xa * yb - xb * ya) / J; /* zeta_z */
                    int64_t g = e * np + l;
                    for (int c = 0; c < 9; c++) C->met[c * C->nl + g] = inv[c];
                    C->met[9 * C->nl + g] = J * C->w[i] * C->w[j] * C->w[k];
                }
    }
    return bad ? -1 : 0;
}

/* Diagonal mass matrix M_I = sum over copies of w_ijk J^e (Eq. (discstrongform)). */
static void build_mass(or_ctx *C)
{
#pragma omp parallel for
    for (int64_t I = 0; I < C->nu; I++) {
        double s = 0.0;
        for (int64_t c = C->off[I]; c < C->off[I + 1]; c++) s += C->met[9 * C->nl + C->cp[c]];
        C->M[I] = s;
    }
}

/*
 * Hydrostatic reference state at unique nodes (reading: the paper's equation
 * set is not in the text; a hydrostatically balanced reference with the
 * perturbation variables rho', u, v, w, theta').
 * Box: isentropic, theta = T0, Exner pi = 1 - g0 z/(cp T0), p = p0 pi^(cp/R),
 *      rho = p/(R T0 pi).
 * Shell: isothermal T0 with g(r) = g0 (a/r)^2: p = p0 exp(-(g0 a/(R T0))(1 - a/r)),
 *      rho = p/(R T0), theta = T0 (p0/p)^(R/cp).
 * In both, p_bar is then re-evaluated from the equation of state
 * p = p0 (R rho theta / p0)^gamma, so that p' is exactly 0 when rho', theta' are 0.
 */
static void build_reference(or_ctx *C)
{
    const or_phys *ph = &C->ph;
    double cv = ph->cp - ph->R, gamma = ph->cp / cv;
    int64_t nu = C->nu;
    for (int64_t I = 0; I < nu; I++) {
        double x = C->xu[I], y = C->xu[nu + I], z = C->xu[2 * nu + I];
        double rb, tb, pcf;
        if (C->m.kind == 0) {
            double pi = 1.0 - ph->g0 * z / (ph->cp * ph->T0);
            pcf = ph->p0 * pow(pi, ph->cp / ph->R);
            rb = pcf / (ph->R * ph->T0 * pi);
            tb = ph->T0;
            C->grav[I] = 0.0; C->grav[nu + I] = 0.0; C->grav[2 * nu + I] = -ph->g0;
        } else {
            /* heights from the radial lattice: 1 - a/r = h/r without cancellation */
            double a = C->m.extent[0];
            double h = C->hu[I], r = a + h;
            pcf = ph->p0 * exp(-(ph->g0 * a / (ph->R * ph->T0)) * (h / r));
            rb = pcf / (ph->R * ph->T0);
            tb = ph->T0 * pow(ph->p0 / pcf, ph->R / ph->cp);
            double gr = ph->g0 * (a / r) * (a / r);
            C->grav[I] = -gr * C->du[I]; C->grav[nu + I] = -gr * C->du[nu + I]; C->grav[2 * nu + I] = -gr * C->du[2 * nu + I];
        }
        C->ref[I] = rb;
        C->ref[nu + I] = tb;
        C->ref[2 * nu + I] = ph->p0 * pow(ph->R * rb * tb / ph->p0, gamma);
    }
}

/*
 * No-flux boundary nodes (reading: the paper does not state the boundary
 * condition): bottom and top radial layers when z is not periodic.
 * Box: top normal +z; bottom normal (-h_x, -h_y, 1)/|.| of the analytic terrain.
 * Shell: radial unit vector at both.
 */
static void build_normals(or_ctx *C)
{
    int64_t nu = C->nu;
    memset(C->nrm, 0, sizeof(double) * 3 * nu);
    memset(C->isbnd, 0, sizeof(int32_t) * nu);
    if (C->m.kind == 0 && C->m.periodic[2]) return;
    for (int64_t I = 0; I < nu; I++) {
        int64_t gk = I / C->nh;
        if (gk != 0 && gk != C->nk - 1) continue;
        double x = C->xu[I], y = C->xu[nu + I], z = C->xu[2 * nu + I];
        double n0, n1, n2;
        if (C->m.kind == 0) {
            if (gk == 0) {
                double Lx = C->m.extent[0], Ly = C->m.extent[1], h0 = C->m.h0;
                double hx = h0 * (2.0 * OR_PI / Lx) * cos(2.0 * OR_PI * x / Lx) * sin(2.0 * OR_PI * y / Ly);
                double hy = h0 * (2.0 * OR_PI / Ly) * sin(2.0 * OR_PI * x / Lx) * cos(2.0 * OR_PI * y / Ly);
                double s = sqrt(hx * hx + hy * hy + 1.0);
                n0 = -hx / s; n1 = -hy / s; n2 = 1.0 / s;
            } else { n0 = 0.0; n1 = 0.0; n2 = 1.0; }
        } else {
            n0 = C->du[I]; n1 = C->du[nu + I]; n2 = C->du[2 * nu + I];
        }
        C->nrm[I] = n0; C->nrm[nu + I] = n1; C->nrm[2 * nu + I] = n2;
        C->isbnd[I] = 1;
    }
}

void or_destroy(or_ctx *C)
{
    if (!C) return;
    free(C->G); free(C->xl); free(C->xu); free(C->met); free(C->M); free(C->ref);
    free(C->grav); free(C->nrm); free(C->isbnd); free(C->off); free(C->cp);
    free(C->dl); free(C->hl); free(C->du); free(C->hu);
    free(C);
}

or_ctx *or_create(const or_mesh_desc *d, const or_phys *ph)
{
    if (check_desc(d)) return NULL;
    or_ctx *C = (or_ctx *)calloc(1, sizeof(or_ctx));
    C->m = *d; C->ph = *ph;
    C->N = d->N; C->P = d->N + 1; C->np = C->P * C->P * C->P;
    or_counts(d, &C->ne, &C->nu, &C->nh);
    C->nl = C->ne * C->np;
    C->nk = C->nu / C->nh;
    C->dtheta = (d->kind == 1);
    or_gll(C->N, C->xi, C->w, C->D);
    C->G = (int32_t *)malloc(sizeof(int32_t) * C->nl);
    C->xl = (double *)malloc(sizeof(double) * 3 * C->nl);
    C->xu = (double *)malloc(sizeof(double) * 3 * C->nu);
    C->met = (double *)malloc(sizeof(double) * 10 * C->nl);
    C->M = (double *)malloc(sizeof(double) * C->nu);
    C->ref = (double *)malloc(sizeof(double) * 3 * C->nu);
    C->grav = (double *)malloc(sizeof(double) * 3 * C->nu);
    C->nrm = (double *)malloc(sizeof(double) * 3 * C->nu);
    C->isbnd = (int32_t *)malloc(sizeof(int32_t) * C->nu);
    C->off = (int64_t *)malloc(sizeof(int64_t) * (C->nu + 1));
    C->cp = (int64_t *)malloc(sizeof(int64_t) * C->nl);
    if (d->kind == 1) {
        C->dl = (double *)malloc(sizeof(double) * 3 * C->nl);
        C->hl = (double *)malloc(sizeof(double) * C->nl);
        C->du = (double *)malloc(sizeof(double) * 3 * C->nu);
        C->hu = (double *)malloc(sizeof(double) * C->nu);
    }
    build_numbering(C);
    build_inverse(C);
    if (build_metric(C)) { or_destroy(C); return NULL; }
    build_mass(C);
    build_reference(C);
    build_normals(C);
    return C;
}

void or_info(const or_ctx *C, int64_t *out /* ne, nl, nu, nh, nk */)
{
    out[0] = C->ne; out[1] = C->nl; out[2] = C->nu; out[3] = C->nh; out[4] = C->nk;
}

/* copy an internal array out: 0 G (int32 [nl]), 1 xl [3][nl], 2 xu [3][nu],
 * 3 metric [10][nl], 4 M [nu], 5 ref [3][nu], 6 gravity [3][nu], 7 normals [3][nu],
 * 8 isbnd (int32 [nu]), 9 gll (xi, w, D) */
int or_get(const or_ctx *C, int what, void *out)
{
    switch (what) {
    case 0: memcpy(out, C->G, sizeof(int32_t) * C->nl); return 0;
    case 1: memcpy(out, C->xl, sizeof(double) * 3 * C->nl); return 0;
    case 2: memcpy(out, C->xu, sizeof(double) * 3 * C->nu); return 0;
    case 3: memcpy(out, C->met, sizeof(double) * 10 * C->nl); return 0;
    case 4: memcpy(out, C->M, sizeof(double) * C->nu); return 0;
    case 5: memcpy(out, C->ref, sizeof(double) * 3 * C->nu); return 0;
    case 6: memcpy(out, C->grav, sizeof(double) * 3 * C->nu); return 0;
    case 7: memcpy(out, C->nrm, sizeof(double) * 3 * C->nu); return 0;
    case 8: memcpy(out, C->isbnd, sizeof(int32_t) * C->nu); return 0;
    case 9: {
        double *o = (double *)out;
        memcpy(o, C->xi, sizeof(double) * C->P);
        memcpy(o + C->P, C->w, sizeof(double) * C->P);
        memcpy(o + 2 * C->P, C->D, sizeof(double) * C->P * C->P);
        return 0;
    }
    default: return -1;
    }
}

/* replace the reference state (for invariance checks on custom backgrounds) */
int or_set(or_ctx *C, int what, const void *in)
{
    switch (what) {
    case 5: memcpy(C->ref, in, sizeof(double) * 3 * C->nu); return 0;
    case 6: memcpy(C->grav, in, sizeof(double) * 3 * C->nu); return 0;
    default: return -1;
    }
}

/* no-flux projection u <- u - (u.n) n at boundary nodes (reading) */
static void project_noflux(const or_ctx *C, double *u, double *v, double *w)
{
    int64_t nu = C->nu;
    for (int64_t I = 0; I < nu; I++) {
        if (!C->isbnd[I]) continue;
        double n0 = C->nrm[I], n1 = C->nrm[nu + I], n2 = C->nrm[2 * nu + I];
        double dn = u[I] * n0 + v[I] * n1 + w[I] * n2;
        u[I] -= dn * n0; v[I] -= dn * n1; w[I] -= dn * n2;
    }
}

/*
 * Initial state at unique nodes (workload definition, not part of the method).
 * q = [5][nu]: rho', u, v, w, theta'.  The potential-temperature perturbation
 * is balanced by rho' = -rho_bar theta'/(theta_bar + theta') so that the
 * pressure is unperturbed.  noise: [3][nu] standard normals or NULL.
 */
int or_init_state(const or_ctx *C, const or_ic_desc *ic, const double *noise, double *q)
{
    int64_t nu = C->nu;
    for (int64_t I = 0; I < nu; I++) {
        double x = C->xu[I], y = C->xu[nu + I], z = C->xu[2 * nu + I];
        double tp = 0.0, u = 0.0, v = 0.0, w = 0.0;
        if (ic->kind == 1) {
            double dx = x - ic->c[0], dy = y - ic->c[1], dz = z - ic->c[2];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            if (r < ic->radius) tp = ic->amp * (1.0 + cos(OR_PI * r / ic->radius)) / 2.0;
        } else if (ic->kind == 2) {
            /* zonal jet and a gaussian blob at great-circle distance d (haversine form) */
            double a = C->m.extent[0];
            double dx0 = C->du[I], dy0 = C->du[nu + I], dz0 = C->du[2 * nu + I];
            double lon = atan2(dy0, dx0), lat = asin(dz0);
            double cl = cos(lat);
            u = ic->jet_u0 * cl * cl * (-sin(lon));
            v = ic->jet_u0 * cl * cl * cos(lon);
            w = 0.0;
            double s1 = sin(0.5 * (lat - ic->c[1])), s2 = sin(0.5 * (lon - ic->c[0]));
            double hv = s1 * s1 + cos(lat) * cos(ic->c[1]) * s2 * s2;
            if (hv > 1.0) hv = 1.0;
            double dist = 2.0 * a * asin(sqrt(hv));
            double hz = (C->hu[I] - ic->c[2]) / ic->lz;
            double hd = dist / ic->radius;
            tp = ic->amp * exp(-hd * hd - hz * hz);
        }
        if (noise) {
            u += ic->noise_amp * noise[I];
            v += ic->noise_amp * noise[nu + I];
            w += ic->noise_amp * noise[2 * nu + I];
        }
        double rb = C->ref[I], tb = C->ref[nu + I];
        q[I] = -rb * tp / (tb + tp);
        q[nu + I] = u; q[2 * nu + I] = v; q[3 * nu + I] = w;
        q[4 * nu + I] = tp;
    }
    project_noflux(C, q + nu, q + 2 * nu, q + 3 * nu);
    return 0;
}

/*
 * Element-wise right-hand side (the paper's create_rhs, Eq. (discstrongform)
 * and Eq. (derivatives)), perturbation form of the inviscid compressible Euler
 * equations with a hydrostatic reference (grad p_bar = rho_bar g):
 *   R_rho'   = -div(rho u)
 *   R_u      = -(u.grad)u - grad(p')/rho + (rho'/rho) g
 *   R_theta' = -u.grad(theta') - u.grad(theta_bar)
 * with rho = rho_bar + rho', and the pressure perturbation from the equation of
 * state p = p0 (R rho theta/p0)^gamma written without cancellation:
 *   Delta = rho' theta_bar + rho_bar theta' + rho' theta',
 *   p' = p_bar expm1(gamma log1p(Delta/(rho_bar theta_bar))).
 * Differentiated nodal fields (all in one pass per direction):
 *   rho u, rho v, rho w, u, v, w, theta', p'  (and theta_bar on the shell).
 * Output: C[v][e][l] = J w_ijk R_v at every element-local node.
 */
static int rhs_impl(const or_ctx *C, const double *q, double *Cout, int scale)
{
    int P = C->P, np = C->np;
    int64_t nu = C->nu, nl = C->nl;
    double cv = C->ph.cp - C->ph.R, gamma = C->ph.cp / cv;
    int nf = C->dtheta ? 9 : 8;
#pragma omp parallel for
    for (int64_t e = 0; e < C->ne; e++) {
        double F[9][OR_MAXP * OR_MAXP * OR_MAXP];
        double rp[OR_MAXP * OR_MAXP * OR_MAXP], rho[OR_MAXP * OR_MAXP * OR_MAXP];
        double U[3][OR_MAXP * OR_MAXP * OR_MAXP], gv[3][OR_MAXP * OR_MAXP * OR_MAXP];
        for (int l = 0; l < np; l++) {
            int64_t I = C->G[e * np + l];
            double r1 = q[I], u = q[nu + I], v = q[2 * nu + I], w = q[3 * nu + I], tp = q[4 * nu + I];
            double rb = C->ref[I], tb = C->ref[nu + I], pb = C->ref[2 * nu + I];
            double rh = rb + r1;
            double dl = r1 * tb + rb * tp + r1 * tp;
            F[0][l] = rh * u; F[1][l] = rh * v; F[2][l] = rh * w;
            F[3][l] = u; F[4][l] = v; F[5][l] = w;
            F[6][l] = tp;
            F[7][l] = pb * expm1(gamma * log1p(dl / (rb * tb)));
            F[8][l] = tb;
            rp[l] = r1; rho[l] = rh;
            U[0][l] = u; U[1][l] = v; U[2][l] = w;
            gv[0][l] = C->grav[I]; gv[1][l] = C->grav[nu + I]; gv[2][l] = C->grav[2 * nu + I];
        }
        for (int k = 0; k < P; k++)
            for (int j = 0; j < P; j++)
                for (int i = 0; i < P; i++) {
                    int l = i + P * (j + P * k);
                    int64_t g = e * np + l;
                    double mx[9];
                    for (int c = 0; c < 9; c++) mx[c] = C->met[c * nl + g];
                    double dx[9], dy[9], dz[9];
                    for (int f = 0; f < nf; f++) {
                        double a = 0.0, b = 0.0, c = 0.0;
                        for (int m = 0; m < P; m++) {
                            a += C->D[i * P + m] * F[f][m + P * (j + P * k)];
                            b += C->D[j * P + m] * F[f][i + P * (m + P * k)];
                            c += C->D[k * P + m] * F[f][i + P * (j + P * m)];
                        }
                        /* chain rule: d/dx = d/dxi xi_x + d/deta eta_x + d/dzeta zeta_x */
                        dx[f] = a * mx[0] + b * mx[3] + c * mx[6];
                        dy[f] = a * mx[1] + b * mx[4] + c * mx[7];
                        dz[f] = a * mx[2] + b * mx[5] + c * mx[8];
                    }
                    double u = U[0][l], v = U[1][l], w = U[2][l];
                    double b = rp[l] / rho[l];
                    double R[5];
                    if (!scale) {
                        R[0] = -(dx[0] + dy[1] + dz[2]);
                        R[1] = -(u * dx[3] + v * dy[3] + w * dz[3]) - dx[7] / rho[l] + b * gv[0][l];
                        R[2] = -(u * dx[4] + v * dy[4] + w * dz[4]) - dy[7] / rho[l] + b * gv[1][l];
                        R[3] = -(u * dx[5] + v * dy[5] + w * dz[5]) - dz[7] / rho[l] + b * gv[2][l];
                        R[4] = -(u * dx[6] + v * dy[6] + w * dz[6]);
                        if (C->dtheta) R[4] -= u * dx[8] + v * dy[8] + w * dz[8];
                    } else {
                        /* magnitudes of the individual terms: the scale that rounding acts on */
                        R[0] = fabs(dx[0]) + fabs(dy[1]) + fabs(dz[2]);
                        R[1] = fabs(u * dx[3]) + fabs(v * dy[3]) + fabs(w * dz[3]) + fabs(dx[7] / rho[l]) + fabs(b * gv[0][l]);
                        R[2] = fabs(u * dx[4]) + fabs(v * dy[4]) + fabs(w * dz[4]) + fabs(dy[7] / rho[l]) + fabs(b * gv[1][l]);
                        R[3] = fabs(u * dx[5]) + fabs(v * dy[5]) + fabs(w * dz[5]) + fabs(dz[7] / rho[l]) + fabs(b * gv[2][l]);
                        R[4] = fabs(u * dx[6]) + fabs(v * dy[6]) + fabs(w * dz[6]);
                        if (C->dtheta) R[4] += fabs(u * dx[8]) + fabs(v * dy[8]) + fabs(w * dz[8]);
                    }
                    double Jw = C->met[9 * nl + g];
                    for (int s = 0; s < 5; s++) Cout[s * nl + g] = Jw * R[s];
                }
    }
    return 0;
}

int or_rhs(const or_ctx *C, const double *q, double *Cout) { return rhs_impl(C, q, Cout, 0); }

/* J w times the sum of the magnitudes of the individual terms of each R
 * (same layout as or_rhs): the conditioning scale of a near-cancelled R. */
int or_rhs_scale(const or_ctx *C, const double *q, double *Cout) { return rhs_impl(C, q, Cout, 1); }

/*
 * Direct stiffness summation (text after Eq. (derivatives)): sum the element
 * contributions at each unique node, gathered over its copies in ascending
 * (e, l) order; flags bit 0: divide by the mass matrix M (weighted by the
 * element volumes); bit 1: no-flux projection of components 1..3 (nvar == 5).
 * cin = [nvar][nl], out = [nvar][nu].
 */
int or_dss(const or_ctx *C, int nvar, const double *cin, int flags, double *out)
{
    int64_t nu = C->nu, nl = C->nl;
#pragma omp parallel for
    for (int64_t I = 0; I < nu; I++) {
        for (int v = 0; v < nvar; v++) {
            double s = 0.0;
            for (int64_t c = C->off[I]; c < C->off[I + 1]; c++) s += cin[v * nl + C->cp[c]];
            if (flags & 1) s = s / C->M[I];
            out[v * nu + I] = s;
        }
    }
    if ((flags & 2) && nvar == 5) project_noflux(C, out + nu, out + 2 * nu, out + 3 * nu);
    return 0;
}

/*
 * SSP-RK3 stage in Shu-Osher form (reading: the paper's five-stage scheme has
 * no coefficients in the text; "update q" of Code example 1):
 *   q_out = a_s qn + b_s (qs + dt R), (a,b) = (0,1), (3/4,1/4), (1/3,2/3).
 */
int or_rk_stage(const or_ctx *C, int stage, double dt, const double *qn, const double *qs, const double *R, double *qout)
{
    int64_t n = 5 * C->nu;
    for (int64_t a = 0; a < n; a++) {
        double y = qs[a] + dt * R[a];
        if (stage == 0) qout[a] = y;
        else if (stage == 1) qout[a] = 0.75 * qn[a] + 0.25 * y;
        else qout[a] = (1.0 / 3.0) * qn[a] + (2.0 / 3.0) * y;
    }
    return 0;
}

/* right-hand side R(q) = DSS_M(create_rhs(q)) with the no-flux projection */
static void full_rhs(const or_ctx *C, const double *q, double *cbuf, double *R)
{
    or_rhs(C, q, cbuf);
    or_dss(C, 5, cbuf, 3, R);
}

/* nsteps SSP-RK3 steps in place on q ([5][nu]); Code example 1 time loop */
int or_step(const or_ctx *C, double dt, int nsteps, double *q)
{
    int64_t n = 5 * C->nu;
    double *cbuf = (double *)malloc(sizeof(double) * 5 * C->nl);
    double *R = (double *)malloc(sizeof(double) * n);
    double *qs = (double *)malloc(sizeof(double) * n);
    if (!cbuf || !R || !qs) { free(cbuf); free(R); free(qs); return -2; }
    for (int s = 0; s < nsteps; s++) {
        full_rhs(C, q, cbuf, R);
        or_rk_stage(C, 0, dt, q, q, R, qs);
        full_rhs(C, qs, cbuf, R);
        or_rk_stage(C, 1, dt, q, qs, R, qs);
        full_rhs(C, qs, cbuf, R);
        or_rk_stage(C, 2, dt, q, qs, R, q);
    }
    free(cbuf); free(R); free(qs);
    return 0;
}

/*
 * The paper's fully explicit scheme has five stages and third order (Sec.
 * "Time Discretization") but the text gives no coefficients.  Reading: the
 * optimal five-stage, third-order strong-stability-preserving Runge-Kutta
 * method of Spiteri and Ruuth (SIAM J. Numer. Anal. 40(2), 2002), in
 * Shu-Osher form
 *   u_0 = q^n,  u_i = sum_{k<i} (alpha_ik u_k + beta_ik dt L(u_k)),  i = 1..5,
 *   q^{n+1} = u_5,
 * with L(u) = DSS_M(create_rhs(u)) as for SSP-RK3.  The nonzero coefficients
 * as published (15 digits); every other alpha_ik, beta_ik is zero.
 */
static const double RK53_ALPHA[6][5] = {
    {0, 0, 0, 0, 0},
    {1.0, 0, 0, 0, 0},
    {0, 1.0, 0, 0, 0},
    {0.355909775063327, 0, 0.644090224936674, 0, 0},
    {0.367933791638137, 0, 0, 0.632066208361863, 0},
    {0, 0, 0.237593836598569, 0, 0.762406163401431},
};
static const double RK53_BETA[6][5] = {
    {0, 0, 0, 0, 0},
    {0.377268915331368, 0, 0, 0, 0},
    {0, 0.377268915331368, 0, 0, 0},
    {0, 0, 0.242995220537396, 0, 0},
    {0, 0, 0, 0.238458932846290, 0},
    {0, 0, 0, 0, 0.287632146308408},
};

/* the tables above, row-major [6][5] each */
void or_rk53_coeffs(double *alpha, double *beta)
{
    for (int i = 0; i < 6; i++)
        for (int k = 0; k < 5; k++) {
            alpha[i * 5 + k] = RK53_ALPHA[i][k];
            beta[i * 5 + k] = RK53_BETA[i][k];
        }
}

/* stage i (1..5) of the Shu-Osher form on n values: out = sum over k < i of
 * alpha_ik U_k + beta_ik dt L_k, where U and L hold u_k and L(u_k) row by row
 * ([6][n] and [5][n]); terms with zero coefficients are skipped */
int or_rk53_combine(int64_t n, int i, double dt, const double *U, const double *L, double *out)
{
    if (i < 1 || i > 5) return -1;
    for (int64_t a = 0; a < n; a++) {
        double s = 0.0;
        for (int k = 0; k < i; k++) {
            if (RK53_ALPHA[i][k] != 0.0) s += RK53_ALPHA[i][k] * U[k * n + a];
            if (RK53_BETA[i][k] != 0.0) s += RK53_BETA[i][k] * dt * L[k * n + a];
        }
        out[a] = s;
    }
    return 0;
}

/* nsteps SSP-RK(5,3) steps in place on q ([5][nu]); every stage value u_k and
 * every L(u_k) is kept for the step */
int or_step_rk53(const or_ctx *C, double dt, int nsteps, double *q)
{
    int64_t n = 5 * C->nu;
    double *cbuf = (double *)malloc(sizeof(double) * 5 * C->nl);
    double *U = (double *)malloc(sizeof(double) * 6 * n);
    double *L = (double *)malloc(sizeof(double) * 5 * n);
    if (!cbuf || !U || !L) { free(cbuf); free(U); free(L); return -2; }
    for (int s = 0; s < nsteps; s++) {
        memcpy(U, q, sizeof(double) * n);
        for (int i = 1; i <= 5; i++) {
            full_rhs(C, U + (i - 1) * n, cbuf, L + (i - 1) * n);
            or_rk53_combine(n, i, dt, U, L, U + i * n);
        }
        memcpy(q, U + 5 * n, sizeof(double) * n);
    }
    free(cbuf); free(U); free(L);
    return 0;
}

/*
 * 1D-IMEX (Sec. "Time Discretization"; Code example 1: "compute IMEX
 * corrections for each vertical column of grid points").  The paper makes
 * implicit corrections along the vertical columns after an explicit leap-frog
 * step and refers the scheme to another paper.  Reading (box with no-flux
 * walls, and the shell):
 *   V(q) is the linearisation about the hydrostatic reference of the terms
 *   that carry vertically propagating sound and gravity, with n the unit
 *   vertical (z on the box, the radial direction on the shell), d/dn = n.grad,
 *   w_n = u.n and s = r^2 on the shell (1 on the box):
 *     V_rho'  = -(1/s) d(s rho_bar w_n)/dn,
 *     V_u     = n (-(1/rho_bar) dp_L/dn + (g.n) rho'/rho_bar),
 *                p_L = (gamma p_bar / rho_bar) (rho' + rho_bar theta'/theta_bar),
 *     V_theta' = -w_n dtheta_bar/dn,
 *   discretised like create_rhs (element-local derivatives through the metric,
 *   J w weighting, DSS and M^-1), the momentum rows set to zero at the walls
 *   (the wall velocity is that of the explicit step);
 *   a step is the leap-frog step with V taken as the trapezoidal mean of the
 *   new and the old level:
 *     q* = q^{n-1} + 2 dt L(q^n)                     (explicit leap-frog)
 *     (I - dt V) q^{n+1} = q* - dt V(2 q^n - q^{n-1})  (vertical correction)
 *   followed by the Robert-Asselin filter with coefficient ra:
 *     q^n <- q^n + ra (q^{n-1} - 2 q^n + q^{n+1}).
 * V couples only the nodes of one vertical lattice line (d/dn acts along
 * zeta: xi and eta are constant along n in both maps), so the correction is
 * one linear solve per line; V changes the velocity only along n.
 */
int or_imex_V(const or_ctx *C, const double *q, double *out)
{
    int P = C->P, np = C->np;
    int64_t nu = C->nu, nl = C->nl;
    int shell = C->m.kind == 1;
    double cv = C->ph.cp - C->ph.R, gamma = C->ph.cp / cv;
    double *cbuf = (double *)malloc(sizeof(double) * 5 * nl);
    if (!cbuf) return -2;
#pragma omp parallel for
    for (int64_t e = 0; e < C->ne; e++) {
        double F[3][OR_MAXP * OR_MAXP * OR_MAXP];
        for (int l = 0; l < np; l++) {
            int64_t I = C->G[e * np + l];
            double rb = C->ref[I], tb = C->ref[nu + I], pb = C->ref[2 * nu + I];
            double n0 = shell ? C->du[I] : 0.0, n1 = shell ? C->du[nu + I] : 0.0, n2 = shell ? C->du[2 * nu + I] : 1.0;
            double r = shell ? C->m.extent[0] + C->hu[I] : 1.0;
            double wn = q[nu + I] * n0 + q[2 * nu + I] * n1 + q[3 * nu + I] * n2;
            F[0][l] = r * r * rb * wn;
            F[1][l] = gamma * pb / rb * (q[I] + rb * q[4 * nu + I] / tb);
            F[2][l] = tb;
        }
        for (int k = 0; k < P; k++)
            for (int j = 0; j < P; j++)
                for (int i = 0; i < P; i++) {
                    int l = i + P * (j + P * k);
                    int64_t g = e * np + l, I = C->G[g];
                    double n[3] = {shell ? C->du[I] : 0.0, shell ? C->du[nu + I] : 0.0, shell ? C->du[2 * nu + I] : 1.0};
                    double r = shell ? C->m.extent[0] + C->hu[I] : 1.0;
                    double dn[3];
                    for (int f = 0; f < 3; f++) {
                        double a = 0.0, b = 0.0, c = 0.0;
                        for (int m = 0; m < P; m++) {
                            a += C->D[i * P + m] * F[f][m + P * (j + P * k)];
                            b += C->D[j * P + m] * F[f][i + P * (m + P * k)];
                            c += C->D[k * P + m] * F[f][i + P * (j + P * m)];
                        }
                        /* n.grad: sum over x, y, z of n_x (d/dxi xi_x + d/deta eta_x + d/dzeta zeta_x) */
                        dn[f] = 0.0;
                        for (int x = 0; x < 3; x++)
                            dn[f] += n[x] * (a * C->met[x * nl + g] + b * C->met[(3 + x) * nl + g] +
                                             c * C->met[(6 + x) * nl + g]);
                    }
                    double rb = C->ref[I];
                    double gn = C->grav[I] * n[0] + C->grav[nu + I] * n[1] + C->grav[2 * nu + I] * n[2];
                    double wn = q[nu + I] * n[0] + q[2 * nu + I] * n[1] + q[3 * nu + I] * n[2];
                    double Vw = -dn[1] / rb + gn * q[I] / rb;
                    double V[5];
                    V[0] = -dn[0] / (r * r);
                    V[1] = Vw * n[0];
                    V[2] = Vw * n[1];
                    V[3] = Vw * n[2];
                    V[4] = -wn * dn[2];
                    double Jw = C->met[9 * nl + g];
                    for (int s = 0; s < 5; s++) cbuf[s * nl + g] = Jw * V[s];
                }
    }
    or_dss(C, 5, cbuf, 1, out);
    for (int64_t I = 0; I < nu; I++)
        if (C->isbnd[I]) out[nu + I] = out[2 * nu + I] = out[3 * nu + I] = 0.0;
    free(cbuf);
    return 0;
}

/* Solve A x = b (n x n, row-major, overwritten) by Gaussian elimination with
 * partial pivoting. */
static int dense_solve(int n, double *A, double *b, double *x)
{
    for (int c = 0; c < n; c++) {
        int piv = c;
        for (int r = c + 1; r < n; r++)
            if (fabs(A[r * n + c]) > fabs(A[piv * n + c])) piv = r;
        if (A[piv * n + c] == 0.0) return -1;
        if (piv != c) {
            for (int k = 0; k < n; k++) {
                double t = A[c * n + k];
                A[c * n + k] = A[piv * n + k];
                A[piv * n + k] = t;
            }
            double t = b[c];
            b[c] = b[piv];
            b[piv] = t;
        }
        for (int r = c + 1; r < n; r++) {
            double f = A[r * n + c] / A[c * n + c];
            if (f == 0.0) continue;
            for (int k = c; k < n; k++) A[r * n + k] -= f * A[c * n + k];
            b[r] -= f * b[c];
        }
    }
    for (int r = n - 1; r >= 0; r--) {
        double s = b[r];
        for (int k = r + 1; k < n; k++) s -= A[r * n + k] * x[k];
        x[r] = s / A[r * n + r];
    }
    return 0;
}

/* the unit vertical at unique node I (z on the box, radial on the shell) */
static void vertical(const or_ctx *C, int64_t I, double *n)
{
    if (C->m.kind == 1) {
        n[0] = C->du[I]; n[1] = C->du[C->nu + I]; n[2] = C->du[2 * C->nu + I];
    } else {
        n[0] = 0.0; n[1] = 0.0; n[2] = 1.0;
    }
}

/* unknown c (0: rho', 1: w_n, 2: theta') of state x at node I */
static double imex_get(const or_ctx *C, const double *x, int c, int64_t I)
{
    int64_t nu = C->nu;
    if (c == 0) return x[I];
    if (c == 2) return x[4 * nu + I];
    double n[3];
    vertical(C, I, n);
    return x[nu + I] * n[0] + x[2 * nu + I] * n[1] + x[3 * nu + I] * n[2];
}

/*
 * nsteps 1D-IMEX leap-frog steps on the pair (q^{n-1}, q^n) in place (after
 * the call qprev holds the filtered last-but-one level and qcur the newest).
 * lines: the vertical lattice lines (horizontal unique index h of the nodes
 * h + n_h k) whose correction is solved, or NULL for all; the rho', velocity
 * and theta' of other lines are set to NaN.  The matrix of V on a line, in the
 * unknowns (rho', w_n, theta') at its levels, is probed with unit states (one
 * at the same level and unknown on every line at once) and each line's system
 * is solved densely; the new velocity is the explicit one with its n
 * component replaced.
 */
int or_imex_step(const or_ctx *C, double dt, double ra, int nsteps, double *qprev, double *qcur,
                 const int32_t *lines, int nlines)
{
    if (C->m.kind == 0 && C->m.periodic[2]) return -3;
    int64_t nu = C->nu, nh = C->nh, nk = C->nk, n5 = 5 * nu;
    int nline = lines ? nlines : (int)nh;
    int nx = 3 * (int)nk;
    double *Vl = (double *)malloc(sizeof(double) * (size_t)nline * nx * nx);
    double *E = (double *)calloc(n5, sizeof(double));
    double *VE = (double *)malloc(sizeof(double) * n5);
    double *cbuf = (double *)malloc(sizeof(double) * 5 * C->nl);
    double *R = (double *)malloc(sizeof(double) * n5);
    double *r = (double *)malloc(sizeof(double) * n5);
    double *sv = (double *)malloc(sizeof(double) * n5);
    double *qn1 = (double *)malloc(sizeof(double) * n5);
    if (!Vl || !E || !VE || !cbuf || !R || !r || !sv || !qn1) {
        free(Vl); free(E); free(VE); free(cbuf); free(R); free(r); free(sv); free(qn1);
        return -2;
    }
    /* column (c, gk) of every line's matrix of V */
    for (int c = 0; c < 3; c++)
        for (int64_t gk = 0; gk < nk; gk++) {
            for (int64_t L = 0; L < nh; L++) {
                int64_t I = L + nh * gk;
                if (c == 0) {
                    E[I] = 1.0;
                } else if (c == 2) {
                    E[4 * nu + I] = 1.0;
                } else {  /* unit vertical velocity */
                    double n[3];
                    vertical(C, I, n);
                    for (int d = 0; d < 3; d++) E[(1 + d) * nu + I] = n[d];
                }
            }
            or_imex_V(C, E, VE);
            memset(E, 0, sizeof(double) * n5);
            for (int a = 0; a < nline; a++) {
                int64_t L = lines ? lines[a] : a;
                for (int c2 = 0; c2 < 3; c2++)
                    for (int64_t k2 = 0; k2 < nk; k2++)
                        Vl[((size_t)a * nx + c2 * nk + k2) * nx + c * nk + gk] = imex_get(C, VE, c2, L + nh * k2);
            }
        }
    for (int st = 0; st < nsteps; st++) {
        full_rhs(C, qcur, cbuf, R);
        for (int64_t a = 0; a < n5; a++) sv[a] = 2.0 * qcur[a] - qprev[a];
        or_imex_V(C, sv, VE);
        /* r = q* - dt V(2 q^n - q^{n-1}),  q* = q^{n-1} + 2 dt L(q^n) */
        for (int64_t a = 0; a < n5; a++) r[a] = (qprev[a] + 2.0 * dt * R[a]) - dt * VE[a];
        memcpy(qn1, r, sizeof(double) * n5);
        if (lines)
            for (int64_t I = 0; I < nu; I++)
                for (int v = 0; v < 5; v++) qn1[v * nu + I] = NAN;
        int fail = 0;
#pragma omp parallel for reduction(| : fail)
        for (int a = 0; a < nline; a++) {
            int64_t L = lines ? lines[a] : a;
            double *A = (double *)malloc(sizeof(double) * nx * nx);
            double *b = (double *)malloc(sizeof(double) * nx);
            double *x = (double *)malloc(sizeof(double) * nx);
            for (int u = 0; u < nx; u++) {
                for (int v = 0; v < nx; v++)
                    A[u * nx + v] = (u == v ? 1.0 : 0.0) - dt * Vl[((size_t)a * nx + u) * nx + v];
                b[u] = imex_get(C, r, u / (int)nk, L + nh * (u % nk));
            }
            fail |= dense_solve(nx, A, b, x);
            for (int64_t k = 0; k < nk; k++) {
                int64_t I = L + nh * k;
                double n[3];
                vertical(C, I, n);
                double rn = imex_get(C, r, 1, I);
                qn1[I] = x[k];
                for (int d = 0; d < 3; d++) qn1[(1 + d) * nu + I] = r[(1 + d) * nu + I] - rn * n[d] + x[nk + k] * n[d];
                qn1[4 * nu + I] = x[2 * nk + k];
            }
            free(A); free(b); free(x);
        }
        if (fail) break;
        for (int64_t a = 0; a < n5; a++) {
            double f = qcur[a] + ra * (qprev[a] - 2.0 * qcur[a] + qn1[a]);
            qprev[a] = f;
            qcur[a] = qn1[a];
        }
    }
    free(Vl); free(E); free(VE); free(cbuf); free(R); free(r); free(sv); free(qn1);
    return 0;
}

/*
 * Boyd-Vandeven filter (Sec. "Filter"; Code example 1: "compute filter",
 * then "DSS and multiply with inverse mass matrix").  The paper names the
 * filter -- a spectral transformation of the element's nodal values that
 * damps the highest modes, i.e. one filter-matrix product per element -- but
 * gives neither its order nor its cutoff.  Reading: the erfc-log form of the
 * Boyd-Vandeven filter with order p and cutoff s as inputs; the modal factor of
 * Legendre mode k is
 *   sigma_k = 1                                   for k <= s,
 *   sigma_k = erfc(2 sqrt(p) chi(t) (t - 1/2)) / 2  with t = (k - s)/(N - s),
 *   chi(t)  = sqrt(-log(1 - 4 (t - 1/2)^2) / (4 (t - 1/2)^2)),  chi(1/2) = 1,
 * so sigma_s = 1 (t = 0, the limit), sigma = 1/2 at t = 1/2 and sigma_N = 0
 * (t = 1).  s >= N leaves the element unchanged.
 */
int or_filter_sigma(int N, double order, int cutoff, double *sigma)
{
    if (N < 1 || N >= OR_MAXP || !(order > 0.0) || cutoff < 0) return -1;
    for (int k = 0; k <= N; k++) {
        if (k < cutoff || cutoff >= N) {
            sigma[k] = 1.0;
            continue;
        }
        double t = (double)(k - cutoff) / (double)(N - cutoff);
        double d = t - 0.5;
        double chi;
        if (t <= 0.0 || t >= 1.0) {   /* the limits of the erfc-log form */
            sigma[k] = t <= 0.0 ? 1.0 : 0.0;
            continue;
        }
        if (d == 0.0) chi = 1.0;
        else chi = sqrt(-log(1.0 - 4.0 * d * d) / (4.0 * d * d));
        sigma[k] = 0.5 * erfc(2.0 * sqrt(order) * chi * d);
    }
    return 0;
}

/* The 1D filter matrix F = V diag(sigma) V^-1 with the Legendre Vandermonde
 * matrix V_ik = P_k(xi_i) at the GLL nodes, V^-1 by Gauss-Jordan elimination
 * with partial pivoting.  F[i*P + m], P = N + 1. */
int or_filter_matrix(int N, double order, int cutoff, double *F)
{
    int P = N + 1;
    double xi[OR_MAXP], w[OR_MAXP], D[OR_MAXP * OR_MAXP], sigma[OR_MAXP];
    double V[OR_MAXP][OR_MAXP], A[OR_MAXP][2 * OR_MAXP];
    if (or_gll(N, xi, w, D) || or_filter_sigma(N, order, cutoff, sigma)) return -1;
    for (int i = 0; i < P; i++)
        for (int k = 0; k < P; k++) {
            double Pk, dPk, Pk1;
            legendre(k, xi[i], &Pk, &dPk, &Pk1);
            V[i][k] = Pk;
        }
    /* [V | I] -> [I | V^-1] */
    for (int i = 0; i < P; i++)
        for (int k = 0; k < 2 * P; k++) A[i][k] = k < P ? V[i][k] : (k - P == i ? 1.0 : 0.0);
    for (int c = 0; c < P; c++) {
        int piv = c;
        for (int r = c + 1; r < P; r++)
            if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
        if (A[piv][c] == 0.0) return -1;
        if (piv != c)
            for (int k = 0; k < 2 * P; k++) {
                double t = A[c][k];
                A[c][k] = A[piv][k];
                A[piv][k] = t;
            }
        double inv = 1.0 / A[c][c];
        for (int k = 0; k < 2 * P; k++) A[c][k] *= inv;
        for (int r = 0; r < P; r++) {
            if (r == c) continue;
            double f = A[r][c];
            for (int k = 0; k < 2 * P; k++) A[r][k] -= f * A[c][k];
        }
    }
    for (int i = 0; i < P; i++)
        for (int m = 0; m < P; m++) {
            double s = 0.0;
            for (int k = 0; k < P; k++) s += V[i][k] * sigma[k] * A[k][P + m];
            F[i * P + m] = s;
        }
    return 0;
}

/*
 * The filter step on the state q ([5][nu], in place): every element's nodal
 * values of each variable are multiplied by the element filter matrix, the
 * Kronecker product F (x) F (x) F of size (N+1)^3 (local node l = i + P(j + P k),
 * so its entry (l, l') is F_ii' F_jj' F_kk'), weighted by J w, summed at the
 * unique nodes and divided by M (or_dss); the velocity is projected at the
 * no-flux walls as after every DSS (reading).  Reading: the filter acts on the
 * perturbation state (rho', u, v, w, theta'), which leaves the hydrostatic
 * reference state untouched.
 */
int or_filter(const or_ctx *C, double order, int cutoff, double *q)
{
    int P = C->P, np = C->np;
    double F[OR_MAXP * OR_MAXP];
    if (or_filter_matrix(C->N, order, cutoff, F)) return -1;
    int64_t nl = C->nl, nu = C->nu;
    double *cbuf = (double *)malloc(sizeof(double) * 5 * nl);
    double *K = (double *)malloc(sizeof(double) * np * np);
    if (!cbuf || !K) { free(cbuf); free(K); return -2; }
    for (int l = 0; l < np; l++) {
        int i = l % P, j = (l / P) % P, k = l / (P * P);
        for (int l2 = 0; l2 < np; l2++) {
            int i2 = l2 % P, j2 = (l2 / P) % P, k2 = l2 / (P * P);
            K[l * np + l2] = F[i * P + i2] * F[j * P + j2] * F[k * P + k2];
        }
    }
#pragma omp parallel for
    for (int64_t e = 0; e < C->ne; e++) {
        double a[OR_MAXP * OR_MAXP * OR_MAXP];
        for (int v = 0; v < 5; v++) {
            for (int l = 0; l < np; l++) a[l] = q[v * nu + C->G[e * np + l]];
            for (int l = 0; l < np; l++) {
                double s = 0.0;
                for (int l2 = 0; l2 < np; l2++) s += K[l * np + l2] * a[l2];
                int64_t c = e * np + l;
                cbuf[v * nl + c] = C->met[9 * nl + c] * s;
            }
        }
    }
    or_dss(C, 5, cbuf, 3, q);
    free(cbuf);
    free(K);
    return 0;
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* threads of the parallel loops from now on (timing only; results do not
 * depend on the thread count) */
void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
