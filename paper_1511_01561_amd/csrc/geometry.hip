// Geometry, reference state and initial state on the device (computed once
// per mesh; the paper computes its metric terms once at the beginning of the
// simulation, remark after Eq. (derivatives)).
#include <cmath>

#include "numa_internal.h"

namespace numa {
namespace {

constexpr double kPi = 3.14159265358979323846;

struct GeoParams {
    int kind, N, P, np;
    int nex, ney, nez;  // elements per direction (shell: ne, ne, nz)
    int walls;
    int64_t ne, nl, nu, nh, nk, ni, nj;
    double L0, L1, L2, h0;  // box: Lx, Ly, H, terrain; shell: a, -, H
    double xi[kMaxP], w[kMaxP], D[kMaxP * kMaxP];
};

GeoParams params(const Mesh &m)
{
    GeoParams g{};
    g.kind = m.d.kind;
    g.N = m.N;
    g.P = m.P;
    g.np = m.np;
    g.nex = m.d.ne[0];
    g.ney = m.d.kind == NUMA_MESH_SHELL ? m.d.ne[0] : m.d.ne[1];
    g.nez = m.d.ne[2];
    g.walls = m.walls ? 1 : 0;
    g.ne = m.ne; g.nl = m.nl; g.nu = m.nu; g.nh = m.nh; g.nk = m.nk; g.ni = m.ni; g.nj = m.nj;
    g.L0 = m.d.extent[0]; g.L1 = m.d.extent[1]; g.L2 = m.d.extent[2]; g.h0 = m.d.terrain_amp;
    for (int i = 0; i < m.P; ++i) { g.xi[i] = m.xi[i]; g.w[i] = m.w[i]; }
    for (int i = 0; i < m.P * m.P; ++i) g.D[i] = m.D[i];
    return g;
}

// Position of lattice index c (0..ncell*N) inside its element, in element
// units: e_c + (1 + xi_{i_c})/2 with e_c clamped to the last element, so every
// copy of a node evaluates the same expression.
__device__ inline double lattice_frac(int64_t c, int N, int ncell, const double *xi)
{
    int64_t e = c / N;
    if (e > ncell - 1) e = ncell - 1;
    int i = (int)(c - (int64_t)N * e);
    return (double)e + (1.0 + xi[i]) / 2.0;
}

__device__ inline void box_xyz(const GeoParams &g, int64_t ci, int64_t cj, int64_t ck, double &x, double &y,
                               double &z)
{
    double xx = g.L0 * lattice_frac(ci, g.N, g.nex, g.xi) / g.nex;
    double yy = g.L1 * lattice_frac(cj, g.N, g.ney, g.xi) / g.ney;
    double zz = g.L2 * lattice_frac(ck, g.N, g.nez, g.xi) / g.nez;
    double h = g.h0 * sin(2.0 * kPi * xx / g.L0) * sin(2.0 * kPi * yy / g.L1);
    x = xx;
    y = yy;
    z = zz + h * (1.0 - zz / g.L2);
}

__device__ inline void face_point(int f, int L, int s, int t, int &X, int &Y, int &Z)
{
    if (f == 0) { X = L; Y = s; Z = t; }
    else if (f == 1) { X = L - s; Y = L; Z = t; }
    else if (f == 2) { X = 0; Y = L - s; Z = t; }
    else if (f == 3) { X = s; Y = 0; Z = t; }
    else if (f == 4) { X = s; Y = t; Z = L; }
    else { X = t; Y = s; Z = 0; }
}

// Equiangular gnomonic node of the surface lattice point (X, Y, Z) at radial
// lattice index ck: unit direction d = P/|P| with P_a = tan(alpha(lattice_a)),
// and height h above the inner radius; the position is (a + h) d.
__device__ inline void shell_node(const GeoParams &g, int X, int Y, int Z, int64_t ck, double d[3], double &h)
{
    int lat[3] = {X, Y, Z};
    double p[3];
    for (int a = 0; a < 3; ++a) {
        double alpha = (kPi / 2.0) * lattice_frac(lat[a], g.N, g.nex, g.xi) / g.nex - kPi / 4.0;
        p[a] = tan(alpha);
    }
    double len = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
    for (int a = 0; a < 3; ++a) d[a] = p[a] / len;
    h = g.L2 * lattice_frac(ck, g.N, g.nez, g.xi) / g.nez;
}

// the shell node of element-local node l of element e
__device__ inline void shell_local(const GeoParams &g, int64_t e, int l, double d[3], double &h)
{
    int i = l % g.P, j = (l / g.P) % g.P, k = l / (g.P * g.P);
    int64_t ex = e % g.nex, ey = (e / g.nex) % g.nex, f = (e / ((int64_t)g.nex * g.nex)) % 6;
    int64_t ez = e / (6 * (int64_t)g.nex * g.nex);
    int X, Y, Z;
    face_point((int)f, g.nex * g.N, (int)(ex * g.N + i), (int)(ey * g.N + j), X, Y, Z);
    shell_node(g, X, Y, Z, ez * g.N + k, d, h);
}

// the shell node of unique node I
__device__ inline void shell_unique(const GeoParams &g, const int32_t *hlat, int64_t I, double d[3], double &h)
{
    int64_t hh = I % g.nh, gk = I / g.nh;
    shell_node(g, hlat[3 * hh], hlat[3 * hh + 1], hlat[3 * hh + 2], gk, d, h);
}

__device__ inline void box_local(const GeoParams &g, int64_t e, int l, double &x, double &y, double &z)
{
    int i = l % g.P, j = (l / g.P) % g.P, k = l / (g.P * g.P);
    int64_t ex = e % g.nex, ey = (e / g.nex) % g.ney, ez = e / ((int64_t)g.nex * g.ney);
    box_xyz(g, ex * g.N + i, ey * g.N + j, ez * g.N + k, x, y, z);
}

__global__ void k_local_coords(GeoParams g, double *X)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.nl) return;
    int64_t e = c / g.np;
    int l = (int)(c - e * g.np);
    double x, y, z;
    if (g.kind == NUMA_MESH_BOX) {
        box_local(g, e, l, x, y, z);
    } else {
        double d[3], h;
        shell_local(g, e, l, d, h);
        double r = g.L0 + h;
        x = r * d[0];
        y = r * d[1];
        z = r * d[2];
    }
    X[c] = x;
    X[g.nl + c] = y;
    X[2 * g.nl + c] = z;
}

// Isoparametric metric of one element per block: A = d(x,y,z)/d(xi,eta,zeta)
// by D contractions of the nodal coordinates, J = det A, inverse = adj(A)/J,
// stored element-major [e][10][np] with J w_i w_j w_k last.  On the shell the
// nodal coordinates are (a + h_k) d_ij and the contractions are taken factor
// by factor (directions along xi and eta, heights along zeta), which is the
// same sum without first rounding the coordinates at the planet's radius.
__global__ void k_metric(GeoParams g, double *met, float *met32, int *bad)
{
    extern __shared__ double sx[];  // [4][np]: x, y, z (box) or d0, d1, d2, h (shell)
    const int64_t e = blockIdx.x;
    const int np = g.np, P = g.P;
    const bool shell = g.kind == NUMA_MESH_SHELL;
    for (int l = threadIdx.x; l < np; l += blockDim.x) {
        if (shell) {
            double d[3], h;
            shell_local(g, e, l, d, h);
            sx[l] = d[0];
            sx[np + l] = d[1];
            sx[2 * np + l] = d[2];
            sx[3 * np + l] = h;
        } else {
            double x, y, z;
            box_local(g, e, l, x, y, z);
            sx[l] = x;
            sx[np + l] = y;
            sx[2 * np + l] = z;
        }
    }
    __syncthreads();
    for (int l = threadIdx.x; l < np; l += blockDim.x) {
        int i = l % P, j = (l / P) % P, k = l / (P * P);
        double A[3][3] = {};
        double hz = 0.0;
        for (int m = 0; m < P; ++m) {
            double di = g.D[i * P + m], dj = g.D[j * P + m], dk = g.D[k * P + m];
            int li = m + P * (j + P * k), lj = i + P * (m + P * k), lk = i + P * (j + P * m);
            for (int a = 0; a < 3; ++a) {
                A[a][0] += di * sx[a * np + li];
                A[a][1] += dj * sx[a * np + lj];
                A[a][2] += dk * sx[a * np + lk];
            }
            if (shell) hz += dk * sx[3 * np + lk];
        }
        if (shell) {
            double r = g.L0 + sx[3 * np + l];
            for (int a = 0; a < 3; ++a) {
                A[a][0] *= r;
                A[a][1] *= r;
                A[a][2] = hz * sx[a * np + l];
            }
        }
        // cofactors
        double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
        double c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
        double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
        double J = A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02;
        if (!(J > 0.0)) atomicOr(bad, 1);
        double inv[10];
        inv[0] = c00 / J;                                         // xi_x
        inv[1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / J;     // xi_y
        inv[2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / J;     // xi_z
        inv[3] = c01 / J;                                         // eta_x
        inv[4] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / J;     // eta_y
        inv[5] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / J;     // eta_z
        inv[6] = c02 / J;                                         // zeta_x
        inv[7] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / J;     // zeta_y
        inv[8] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / J;     // zeta_z
        inv[9] = J * (g.w[i] * g.w[j] * g.w[k]);
        double *o = met + e * 10 * np + l;
        for (int c = 0; c < 10; ++c) o[c * np] = inv[c];
        if (met32) {
            float *o32 = met32 + e * 10 * np + l;
            for (int c = 0; c < 10; ++c) o32[c * np] = (float)inv[c];
        }
    }
}

// M_I = sum over the copies of J w (ascending element-local order), and 1/M.
__global__ void k_mass(GeoParams g, const int32_t *off, const int32_t *idx, const double *met, double *M,
                       double *Minv)
{
    int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= g.nu) return;
    double s = 0.0;
    for (int32_t c = off[I]; c < off[I + 1]; ++c) {
        int64_t cc = idx[c];
        int64_t e = cc / g.np;
        int l = (int)(cc - e * g.np);
        s += met[(e * 10 + 9) * g.np + l];
    }
    M[I] = s;
    Minv[I] = 1.0 / s;
}

// Inverse mass of the recomputed metric: per unique node, the sum over its
// copies (ascending, as k_mass) of the J w that the recomputed-metric element
// kernels form, the same products: box c0 w_k (column factor c0 of the
// element's (i, j) column), shell (column factor 9) x (layer factor 2).
__global__ void k_mass_recomputed(GeoParams g, const int32_t *off, const int32_t *idx, const double *hcol,
                                  const double *scol, const double *slay, double *MinvR)
{
    int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= g.nu) return;
    const int PP = g.P * g.P;
    double s = 0.0;
    for (int32_t c = off[I]; c < off[I + 1]; ++c) {
        const int64_t cc = idx[c];
        const int64_t e = cc / g.np;
        const int l = (int)(cc - e * g.np), ij = l % PP, k = l / PP;
        if (g.kind == NUMA_MESH_BOX) {
            const int64_t ex = e % g.nex, ey = (e / g.nex) % g.ney;
            s += hcol[(ex + g.nex * ey) * (4 * PP) + ij] * g.w[k];
        } else {
            const int64_t neh = 6 * (int64_t)g.nex * g.nex, eh = e % neh, ez = e / neh;
            s += scol[eh * (13 * PP) + 9 * PP + ij] * slay[4 * (ez * g.P + k) + 2];
        }
    }
    MinvR[I] = 1.0 / s;
}

// lean workspace: M and M^-1 from the recomputed J w (the stored metric is
// not kept)
__global__ void k_mass_from_recomputed(GeoParams g, const double *MinvR, double *M, double *Minv)
{
    int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= g.nu) return;
    M[I] = 1.0 / MinvR[I];
    Minv[I] = MinvR[I];
}

__global__ void k_unique_coords(GeoParams g, const int32_t *hlat, double *xu)
{
    int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= g.nu) return;
    double x, y, z;
    if (g.kind == NUMA_MESH_BOX) {
        int64_t gi = I % g.ni, gj = (I / g.ni) % g.nj, gk = I / (g.ni * g.nj);
        box_xyz(g, gi, gj, gk, x, y, z);
    } else {
        double d[3], h;
        shell_unique(g, hlat, I, d, h);
        double r = g.L0 + h;
        x = r * d[0];
        y = r * d[1];
        z = r * d[2];
    }
    xu[I] = x;
    xu[g.nu + I] = y;
    xu[2 * g.nu + I] = z;
}

// Hydrostatic reference (isentropic box, isothermal shell with g = g0 (a/r)^2);
// p_bar re-evaluated from the equation of state so that p' = 0 at rest.
__global__ void k_reference(GeoParams g, numa_phys ph, const int32_t *hlat, const double *xu, double *ref,
                            double *grav)
{
    int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= g.nu) return;
    double z = xu[2 * g.nu + I];
    double gamma = ph.cp / (ph.cp - ph.R);
    double rb, tb;
    if (g.kind == NUMA_MESH_BOX) {
        double exner = 1.0 - ph.g0 * z / (ph.cp * ph.T0);
        double pcf = ph.p0 * pow(exner, ph.cp / ph.R);
        rb = pcf / (ph.R * ph.T0 * exner);
        tb = ph.T0;
    } else {
        // height from the radial lattice: 1 - a/r = h/r without cancellation
        double d[3], h;
        shell_unique(g, hlat, I, d, h);
        double a = g.L0, r = a + h;
        double pcf = ph.p0 * exp(-(ph.g0 * a / (ph.R * ph.T0)) * (h / r));
        rb = pcf / (ph.R * ph.T0);
        tb = ph.T0 * pow(ph.p0 / pcf, ph.R / ph.cp);
        double gr = ph.g0 * (a / r) * (a / r);
        grav[I] = -gr * d[0];
        grav[g.nu + I] = -gr * d[1];
        grav[2 * g.nu + I] = -gr * d[2];
    }
    ref[I] = rb;
    ref[g.nu + I] = tb;
    ref[2 * g.nu + I] = ph.p0 * pow(ph.R * rb * tb / ph.p0, gamma);
}

// Wall normals of the bottom and top layers: [2][3][nh].
__global__ void k_normals(GeoParams g, const int32_t *hlat, const double *xu, double *nrm)
{
    int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= g.nh) return;
    for (int side = 0; side < 2; ++side) {
        int64_t I = side == 0 ? h : (g.nk - 1) * g.nh + h;
        double x = xu[I], y = xu[g.nu + I];
        double n[3];
        if (g.kind == NUMA_MESH_BOX) {
            if (side == 0) {
                double hx = g.h0 * (2.0 * kPi / g.L0) * cos(2.0 * kPi * x / g.L0) * sin(2.0 * kPi * y / g.L1);
                double hy = g.h0 * (2.0 * kPi / g.L1) * sin(2.0 * kPi * x / g.L0) * cos(2.0 * kPi * y / g.L1);
                double s = sqrt(hx * hx + hy * hy + 1.0);
                n[0] = -hx / s; n[1] = -hy / s; n[2] = 1.0 / s;
            } else {
                n[0] = 0.0; n[1] = 0.0; n[2] = 1.0;
            }
        } else {
            double hh;
            shell_unique(g, hlat, I, n, hh);
        }
        for (int a = 0; a < 3; ++a) nrm[(side * 3 + a) * g.nh + h] = n[a];
    }
}

__global__ void k_init_state(GeoParams g, numa_ic ic, const int32_t *hlat, const double *xu, const double *ref,
                             const double *nrm, const double *noise, double *q)
{
    int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= g.nu) return;
    double x = xu[I], y = xu[g.nu + I], z = xu[2 * g.nu + I];
    double tp = 0.0, u = 0.0, v = 0.0, w = 0.0;
    if (ic.kind == 1) {
        double dx = x - ic.c[0], dy = y - ic.c[1], dz = z - ic.c[2];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        if (r < ic.radius) tp = ic.amp * (1.0 + cos(kPi * r / ic.radius)) / 2.0;
    } else if (ic.kind == 2) {
        // zonal jet and a gaussian blob at great-circle distance (haversine form)
        double d[3], h;
        shell_unique(g, hlat, I, d, h);
        double a = g.L0;
        double lon = atan2(d[1], d[0]), lat = asin(d[2]);
        double cl = cos(lat);
        u = ic.jet_u0 * cl * cl * (-sin(lon));
        v = ic.jet_u0 * cl * cl * cos(lon);
        double s1 = sin(0.5 * (lat - ic.c[1])), s2 = sin(0.5 * (lon - ic.c[0]));
        double hv = fmin(1.0, s1 * s1 + cos(lat) * cos(ic.c[1]) * s2 * s2);
        double hd = 2.0 * a * asin(sqrt(hv)) / ic.radius;
        double hz = (h - ic.c[2]) / ic.lz;
        tp = ic.amp * exp(-hd * hd - hz * hz);
    }
    if (noise) {
        u += ic.noise_amp * noise[I];
        v += ic.noise_amp * noise[g.nu + I];
        w += ic.noise_amp * noise[2 * g.nu + I];
    }
    if (g.walls && (I < g.nh || I >= g.nu - g.nh)) {
        int side = I < g.nh ? 0 : 1;
        int64_t h = side == 0 ? I : I - (g.nu - g.nh);
        double n0 = nrm[(side * 3) * g.nh + h], n1 = nrm[(side * 3 + 1) * g.nh + h], n2 = nrm[(side * 3 + 2) * g.nh + h];
        double dn = u * n0 + v * n1 + w * n2;
        u -= dn * n0; v -= dn * n1; w -= dn * n2;
    }
    double rb = ref[I], tb = ref[g.nu + I];
    q[I] = -rb * tp / (tb + tp);
    q[g.nu + I] = u;
    q[2 * g.nu + I] = v;
    q[3 * g.nu + I] = w;
    q[4 * g.nu + I] = tp;
}

__global__ void k_export_metric(GeoParams g, const double *met, double *out)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.nl) return;
    int64_t e = c / g.np;
    int l = (int)(c - e * g.np);
    for (int a = 0; a < 10; ++a) out[a * g.nl + c] = met[(e * 10 + a) * g.np + l];
}

__global__ void k_box_gravity(GeoParams g, double g0, double *out)
{
    int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= g.nu) return;
    out[I] = 0.0;
    out[g.nu + I] = 0.0;
    out[2 * g.nu + I] = -g0;
}

// Column factors of the recomputed box metric.  The map x = x(xi),
// y = y(eta), z' = z(zeta) + h(x, y)(1 - z/H) has x_xi = Lx/(2 nx),
// y_eta = Ly/(2 ny), z_zeta = (1 - h/H) H/(2 nz), z_xi = (1 - z/H) dh/dxi and
// z_eta = (1 - z/H) dh/deta, so at local (i, j) of element column (ex, ey)
//   c0 = x_xi y_eta z_zeta w_i w_j         (J w_ijk = c0 w_k)
//   c1 = 1/z_zeta                          (zeta_z)
//   c2 = -(dh/dxi)/(x_xi z_zeta)           (zeta_x = (1 - z/H) c2)
//   c3 = -(dh/deta)/(y_eta z_zeta)         (zeta_y = (1 - z/H) c3)
// with h as in box_xyz, dh/dxi = sum_m D_im h_mj and dh/deta = sum_m D_jm h_im;
// xi_x = 1/x_xi and eta_y = 1/y_eta, the other entries are zero.  Layout
// [nx*ny][4][(N+1)^2], column ex + nx*ey: the per-node metric then takes no
// division and no transcendental.
__device__ inline double box_terrain(const GeoParams &g, int64_t ci, int64_t cj)
{
    const double xx = g.L0 * lattice_frac(ci, g.N, g.nex, g.xi) / g.nex;
    const double yy = g.L1 * lattice_frac(cj, g.N, g.ney, g.xi) / g.ney;
    return g.h0 * sin(2.0 * kPi * xx / g.L0) * sin(2.0 * kPi * yy / g.L1);
}

__global__ void k_box_columns(GeoParams g, double *hcol, int *bad)
{
    const int PP = g.P * g.P;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)g.nex * g.ney * PP) return;
    const int64_t col = t / PP;
    const int l = (int)(t - col * PP), i = l % g.P, j = l / g.P;
    const int64_t ex = col % g.nex, ey = col / g.nex;
    const int64_t ci = ex * g.N, cj = ey * g.N;
    double hx = 0.0, hy = 0.0;
    for (int m = 0; m < g.P; ++m) {
        hx += g.D[i * g.P + m] * box_terrain(g, ci + m, cj + j);
        hy += g.D[j * g.P + m] * box_terrain(g, ci + i, cj + m);
    }
    const double h = box_terrain(g, ci + i, cj + j);
    const double xa = g.L0 / (2.0 * g.nex), yb = g.L1 / (2.0 * g.ney);
    const double zc = (1.0 - h / g.L2) * (g.L2 / (2.0 * g.nez));
    if (!(zc > 0.0)) *bad = 1;  // the terrain reaches the top: no positive Jacobian
    double *o = hcol + col * 4 * PP + l;
    o[0] = xa * yb * zc * (g.w[i] * g.w[j]);
    o[PP] = 1.0 / zc;
    o[2 * PP] = -hx / (xa * zc);
    o[3 * PP] = -hy / (yb * zc);
}

// Column and layer factors of the recomputed shell metric.  The map
// x = (a + h(zeta)) d(xi, eta) with the isoparametric contractions of k_metric
// gives the columns A = [r d_xi, r d_eta, h_zeta d] (r = a + h, d_xi =
// sum_m D_im d_mj, d_eta = sum_m D_jm d_im, h_zeta = sum_m D_km h_m), so with
// T = d_xi . (d_eta x d):
//   grad xi = (d_eta x d)/(r T), grad eta = (d x d_xi)/(r T),
//   grad zeta = (d_xi x d_eta)/(h_zeta T), J w = T w_i w_j r^2 h_zeta w_k.
// Per element column (horizontal element eh, local (i, j)), layout
// [6 ne^2][13][(N+1)^2]: (d_eta x d)/T (3), (d x d_xi)/T (3), (d_xi x d_eta)/T
// (3), T w_i w_j, d (3, for gravity).  Per radial node (layer ez, local k),
// layout [nz (N+1)][4]: 1/r, 1/h_zeta, r^2 h_zeta w_k, g0 (a/r)^2.  The
// horizontal unique id of each column is its bottom node's id.
__global__ void k_shell_columns(GeoParams g, const int32_t *G, double *scol, int32_t *shid)
{
    const int PP = g.P * g.P;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 6 * (int64_t)g.nex * g.nex * PP) return;
    const int64_t eh = t / PP;
    const int c = (int)(t - eh * PP), i = c % g.P, j = c / g.P;
    double d[3], h, dx[3] = {0, 0, 0}, dy[3] = {0, 0, 0};
    for (int m = 0; m < g.P; ++m) {
        double dm[3];
        shell_local(g, eh, m + g.P * j, dm, h);
        for (int a = 0; a < 3; ++a) dx[a] += g.D[i * g.P + m] * dm[a];
        shell_local(g, eh, i + g.P * m, dm, h);
        for (int a = 0; a < 3; ++a) dy[a] += g.D[j * g.P + m] * dm[a];
    }
    shell_local(g, eh, c, d, h);
    const double u1[3] = {dy[1] * d[2] - dy[2] * d[1], dy[2] * d[0] - dy[0] * d[2], dy[0] * d[1] - dy[1] * d[0]};
    const double u2[3] = {d[1] * dx[2] - d[2] * dx[1], d[2] * dx[0] - d[0] * dx[2], d[0] * dx[1] - d[1] * dx[0]};
    const double u3[3] = {dx[1] * dy[2] - dx[2] * dy[1], dx[2] * dy[0] - dx[0] * dy[2], dx[0] * dy[1] - dx[1] * dy[0]};
    const double T = dx[0] * u1[0] + dx[1] * u1[1] + dx[2] * u1[2];
    double *o = scol + eh * 13 * PP + c;
    for (int a = 0; a < 3; ++a) {
        o[a * PP] = u1[a] / T;
        o[(3 + a) * PP] = u2[a] / T;
        o[(6 + a) * PP] = u3[a] / T;
        o[(10 + a) * PP] = d[a];
    }
    o[9 * PP] = T * (g.w[i] * g.w[j]);
    shid[t] = G[eh * g.np + c];  // element eh of the bottom layer, local node (i, j, 0)
}

__global__ void k_shell_layers(GeoParams g, double g0, double *slay)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)g.nez * g.P) return;
    const int64_t ez = t / g.P;
    const int k = (int)(t - ez * g.P);
    double d[3], h, hz = 0.0;
    const int64_t e0 = ez * 6 * (int64_t)g.nex * g.nex;  // any element of layer ez
    for (int m = 0; m < g.P; ++m) {
        shell_local(g, e0, g.P * g.P * m, d, h);
        hz += g.D[k * g.P + m] * h;
    }
    shell_local(g, e0, g.P * g.P * k, d, h);
    const double r = g.L0 + h, ar = g.L0 / r;
    slay[4 * t] = 1.0 / r;
    slay[4 * t + 1] = 1.0 / hz;
    slay[4 * t + 2] = r * r * hz * g.w[k];
    slay[4 * t + 3] = g0 * ar * ar;
}

inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

int32_t launch_geometry(Mesh &m, hipStream_t s)
{
    GeoParams g = params(m);
    DeviceView &v = m.dv;
    if (!m.uploaded) {
        if (v.G) NUMA_HIP(hipMemcpyAsync(v.G, m.G.data(), 4 * m.nl, hipMemcpyHostToDevice, s));
        NUMA_HIP(hipMemcpyAsync(v.off, m.off.data(), 4 * (m.nu + 1), hipMemcpyHostToDevice, s));
        NUMA_HIP(hipMemcpyAsync(v.idx, m.idx.data(), 4 * m.nl, hipMemcpyHostToDevice, s));
        if (v.hlat) NUMA_HIP(hipMemcpyAsync(v.hlat, m.hlat.data(), 12 * m.nh, hipMemcpyHostToDevice, s));
        if (v.hoff) {
            NUMA_HIP(hipMemcpyAsync(v.hoff, m.hoff.data(), 4 * m.hoff.size(), hipMemcpyHostToDevice, s));
            NUMA_HIP(hipMemcpyAsync(v.hidx, m.hidx.data(), 4 * m.hidx.size(), hipMemcpyHostToDevice, s));
        }
        if (v.own) {
            NUMA_HIP(hipMemcpyAsync(v.own, m.own.data(), 4 * m.nu, hipMemcpyHostToDevice, s));
            NUMA_HIP(hipMemcpyAsync(v.toff, m.toff.data(), 4 * (m.nu + 1), hipMemcpyHostToDevice, s));
            NUMA_HIP(hipMemcpyAsync(v.tidx, m.tidx.data(), 4 * m.nl, hipMemcpyHostToDevice, s));
        }
        m.D32.assign(m.D, m.D + m.P * m.P);
        NUMA_HIP(hipMemcpyAsync(v.D64, m.D, 8 * m.P * m.P, hipMemcpyHostToDevice, s));
        NUMA_HIP(hipMemcpyAsync(v.D32, m.D32.data(), 4 * m.P * m.P, hipMemcpyHostToDevice, s));
        NUMA_HIP(hipMemcpyAsync(v.xi64, m.xi, 8 * m.P, hipMemcpyHostToDevice, s));
        NUMA_HIP(hipMemcpyAsync(v.w64, m.w, 8 * m.P, hipMemcpyHostToDevice, s));
        // the pageable-memory copies above must finish before the host vectors can change
        NUMA_HIP(hipStreamSynchronize(s));
        m.uploaded = true;
    }
    const int bs = 256;
    int *bad = v.flag;
    NUMA_HIP(hipMemsetAsync(bad, 0, sizeof(int), s));
    if (v.met) {  // not in a lean workspace: the mass then comes from the recomputed J w below
        int mt = ((m.np + 63) / 64) * 64;
        if (mt > 256) mt = 256;
        hipLaunchKernelGGL(k_metric, dim3((unsigned)m.ne), dim3(mt), 4 * m.np * sizeof(double), s, g, v.met,
                           v.met32, bad);
        hipLaunchKernelGGL(k_mass, dim3(nblocks(m.nu, bs)), dim3(bs), 0, s, g, v.off, v.idx, v.met, v.M, v.Minv);
    }
    hipLaunchKernelGGL(k_unique_coords, dim3(nblocks(m.nu, bs)), dim3(bs), 0, s, g, v.hlat, v.xu);
    hipLaunchKernelGGL(k_reference, dim3(nblocks(m.nu, bs)), dim3(bs), 0, s, g, m.ph, v.hlat, v.xu, v.ref, v.grav);
    hipLaunchKernelGGL(k_normals, dim3(nblocks(m.nh, bs)), dim3(bs), 0, s, g, v.hlat, v.xu, v.nrm);
    if (v.hcol)
        hipLaunchKernelGGL(k_box_columns, dim3(nblocks((int64_t)g.nex * g.ney * m.P * m.P, bs)), dim3(bs), 0, s, g,
                           v.hcol, bad);
    if (v.scol) {
        hipLaunchKernelGGL(k_shell_columns, dim3(nblocks(6 * (int64_t)g.nex * g.nex * m.P * m.P, bs)), dim3(bs), 0, s,
                           g, v.G, v.scol, v.shid);
        hipLaunchKernelGGL(k_shell_layers, dim3(nblocks((int64_t)g.nez * m.P, bs)), dim3(bs), 0, s, g, m.ph.g0,
                           v.slay);
    }
    hipLaunchKernelGGL(k_mass_recomputed, dim3(nblocks(m.nu, bs)), dim3(bs), 0, s, g, v.off, v.idx, v.hcol, v.scol,
                       v.slay, v.MinvR);
    if (!v.met)
        hipLaunchKernelGGL(k_mass_from_recomputed, dim3(nblocks(m.nu, bs)), dim3(bs), 0, s, g, v.MinvR, v.M, v.Minv);
    NUMA_HIP(hipGetLastError());
    int hbad = 0;
    NUMA_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    NUMA_HIP(hipStreamSynchronize(s));
    if (hbad) {
        set_error("geometry: non-positive Jacobian");
        return NUMA_EINVAL;
    }
    return NUMA_OK;
}

int32_t launch_export(Mesh &m, int32_t what, void *out, hipStream_t s)
{
    GeoParams g = params(m);
    DeviceView &v = m.dv;
    const int bs = 256;
    switch (what) {
    case NUMA_FIELD_MASS:
        NUMA_HIP(hipMemcpyAsync(out, v.M, 8 * m.nu, hipMemcpyDeviceToDevice, s));
        break;
    case NUMA_FIELD_REF:
        NUMA_HIP(hipMemcpyAsync(out, v.ref, 24 * m.nu, hipMemcpyDeviceToDevice, s));
        break;
    case NUMA_FIELD_COORDS:
        NUMA_HIP(hipMemcpyAsync(out, v.xu, 24 * m.nu, hipMemcpyDeviceToDevice, s));
        break;
    case NUMA_FIELD_METRIC:
        if (!v.met) {
            set_error("export: the per-node metric is not kept in a lean workspace (NUMA_WS_LEAN)");
            return NUMA_ENOMEM;
        }
        hipLaunchKernelGGL(k_export_metric, dim3(nblocks(m.nl, bs)), dim3(bs), 0, s, g, v.met, (double *)out);
        break;
    case NUMA_FIELD_GRAVITY:
        if (v.grav) NUMA_HIP(hipMemcpyAsync(out, v.grav, 24 * m.nu, hipMemcpyDeviceToDevice, s));
        else hipLaunchKernelGGL(k_box_gravity, dim3(nblocks(m.nu, bs)), dim3(bs), 0, s, g, m.ph.g0, (double *)out);
        break;
    case NUMA_FIELD_LOCAL_COORDS:
        hipLaunchKernelGGL(k_local_coords, dim3(nblocks(m.nl, bs)), dim3(bs), 0, s, g, (double *)out);
        break;
    default:
        set_error("export: unknown field %d", what);
        return NUMA_EINVAL;
    }
    NUMA_HIP(hipGetLastError());
    return NUMA_OK;
}

int32_t launch_init_state(Mesh &m, const numa_ic &ic, const double *noise, double *q, hipStream_t s)
{
    GeoParams g = params(m);
    const int bs = 256;
    hipLaunchKernelGGL(k_init_state, dim3(nblocks(m.nu, bs)), dim3(bs), 0, s, g, ic, m.dv.hlat, m.dv.xu, m.dv.ref,
                       m.dv.nrm, noise, q);
    NUMA_HIP(hipGetLastError());
    return NUMA_OK;
}

}  // namespace numa
