// Device code shared by the single-mesh and the batched kernels: the per-node
// element right-hand side, the wall projection, the stage combination and the
// per-node finish of a fused stage on the box.  Included by the .hip sources.
#pragma once

#include <cmath>
#include <type_traits>

#include "numa_internal.h"

namespace numa {
namespace dev {

// Per-mesh constants of the recomputed box metric: xi_x = 2 nx/Lx,
// eta_y = 2 ny/Ly and 1/nz (the undeformed level z/H of a node is
// (ez + (1 + xi_k)/2)/nz).  Everything that varies over the terrain comes
// from the column table (Mesh workspace hcol).
struct BoxMetric {
    double ixa, iyb, inz;
};

// (1 + x)^gamma - 1 by its binomial series sum_k c_k x^k, c_1 = gamma,
// c_{k+1} = c_k (gamma - k)/(k + 1), used for |x| < 1/64 where ten terms leave a
// truncation error below 1e-19 relative (|c_11| |x|^11 < 1e-22 against
// |(1 + x)^gamma - 1| > 0.01 |x| for gamma in (1, 2]); otherwise
// expm1(gamma log1p(x)).  This is the pressure perturbation of the equation of
// state p = p0 (R rho theta / p0)^gamma about the reference, without cancellation.
constexpr int kEosTerms = 10;
// The rarely taken branch is a separate function: inlined, the constants of
// log1p and expm1 would be hoisted out of the kernels' loops and held in
// registers for the whole kernel.
__device__ __noinline__ double eos_rel_large(double x, double gamma) { return expm1(gamma * log1p(x)); }
__device__ __forceinline__ double eos_rel(double x, double gamma, const double *c)
{
    if (fabs(x) < 0.015625) {
        double r = c[kEosTerms - 1];
#pragma unroll
        for (int k = kEosTerms - 2; k >= 0; --k) r = r * x + c[k];
        return r * x;
    }
    return eos_rel_large(x, gamma);
}

// host: constants of the recomputed metric of a box mesh
inline BoxMetric box_metric(const Mesh &m)
{
    BoxMetric b;
    b.ixa = 1.0 / (m.d.extent[0] / (2.0 * m.d.ne[0]));
    b.iyb = 1.0 / (m.d.extent[1] / (2.0 * m.d.ne[1]));
    b.inz = 1.0 / m.d.ne[2];
    return b;
}

inline void eos_coeffs(double gamma, double *c)
{
    c[0] = gamma;
    for (int k = 1; k < kEosTerms; ++k) c[k] = c[k - 1] * (gamma - k) / (k + 1);
}

template <typename T>
struct RhsArgs {
    const int32_t *G;  // gather map (shell); the box computes unique ids from its lattice
    const double *q, *ref, *grav;
    const T *met;
    const T *D;
    const double *hcol;  // box: column factors of the recomputed metric
    int64_t nl, nu;
    double gamma, g0;
    int nx, ny, nz;      // box: elements along x, y, z
    int ni, nj, nk;      // box: lattice extents (x, y periodic; nk = -1 unless z is)
    FastDiv fx, fy;      // box: division by nx and ny
    const double *scol, *slay;  // shell, recomputed metric: column and layer factors
    const int32_t *shid;        // shell, recomputed metric: horizontal unique id of each column
    int64_t nh;                 // shell: horizontal nodes
    FastDiv feh;                // shell: division by the elements of one layer (6 ne^2)
    const double *xi, *w, *Dd;  // FP64 GLL nodes, weights, derivative matrix
    BoxMetric bm;               // box: constants of the recomputed metric
    double eos[kEosTerms];      // coefficients of the binomial series of (1 + x)^gamma - 1
    double cdt;                 // shell stage (fold != 0): the stage's cdt
    int fold;                   // shell stage: J w (q_s + cdt R) away from the walls (k_shell_finish)
};

// Metric of a box element: stored per node (the general path), or recomputed
// from the terrain-following map z' = z + h(x, y)(1 - z/H).
enum { kMetricStored = 0, kMetricBox = 1, kMetricShell = 2 };

// coordinates of box element e = ex + nx (ey + ny ez)
struct BoxElem {
    int ex, ey, ez;
};

__device__ __forceinline__ BoxElem box_elem(uint32_t e, const FastDiv &fx, const FastDiv &fy)
{
    const uint32_t t = fdiv(e, fx), ez = fdiv(t, fy);
    return BoxElem{(int)(e - t * fx.d), (int)(t - ez * fy.d), (int)ez};
}

// unique id of local node (i, j, k) of box element b: the element's lattice
// corner plus the local offset, wrapped in the periodic directions
template <int N, typename T>
__device__ __forceinline__ int32_t box_unique(const RhsArgs<T> &a, const BoxElem &b, int i, int j, int k)
{
    int gi = b.ex * N + i, gj = b.ey * N + j, gk = b.ez * N + k;
    if (gi == a.ni) gi = 0;
    if (gj == a.nj) gj = 0;
    if (gk == a.nk) gk = 0;
    return gi + a.ni * (gj + a.nj * gk);
}

template <int N>
constexpr int block_threads() { return (((N + 1) * (N + 1) * (N + 1) + 63) / 64) * 64; }

// Per-node result of the element RHS.
template <typename T>
struct NodeOut {
    T R[5];  // R_rho', R_u, R_v, R_w, R_theta'
    T Jw;
};

// Operands of node l that are loaded before its element's tile is built:
// state, reference, and the metric (stored) or the column factors (recomputed).
template <typename T>
struct NodeIn {
    double rp, u, v, w, tp, rb, tb, pb;
    double c0, c1, c2, c3, zk;  // box, recomputed metric: column factors (c0 with w_k), xi_k
    T mx[10];                   // stored metric and shell: inverse metric (9) and J w
    T gv[3];                    // shell, recomputed metric: gravity
    int32_t I;                  // unique id
    int32_t I0;                 // shell, recomputed metric: unique id of the element's first node
    int ez;                     // box: element layer
};

// The three phases of the element right-hand side at node l of element e:
// node_gather issues the loads, node_stage evaluates the equation of state
// and writes the node's fields into the element tile, node_derive (after a
// barrier) differentiates the tile and evaluates R.  element_rhs runs them in
// order.
//
// GEO == kMetricBox (box meshes): the isoparametric metric of the
// terrain-following map x = x(xi), y = y(eta), z' = z(zeta) + h(x, y)(1 - z/H)
// is computed instead of read: with the node's column factors c0..c3 (see
// k_box_columns) and its undeformed level z/H, xi_x = 2 nx/Lx,
// eta_y = 2 ny/Ly, zeta = ((1 - z/H) c2, (1 - z/H) c3, c1), J w = c0 w_k, all
// other entries zero.
template <int N, typename T, bool SHELL, int GEO>
__device__ __forceinline__ void node_gather(const RhsArgs<T> &a, int64_t e, int l, NodeIn<T> &in)
{
    constexpr int P = N + 1, PP = P * P, NP = PP * P;
    if (l >= NP) return;
    const int i = l % P, j = (l / P) % P, k = l / PP;
    if constexpr (SHELL && GEO == kMetricShell) {
        // the column's horizontal id plus the radial layer; metric and gravity
        // from the column and layer factors (k_shell_columns, k_shell_layers)
        const uint32_t ez = fdiv((uint32_t)e, a.feh);
        const int64_t eh = e - (int64_t)ez * a.feh.d;
        const int c = i + P * j;
        const int32_t *hp = a.shid + eh * PP;
        in.I = hp[c] + (int32_t)(a.nh * ((int64_t)ez * N + k));
        in.I0 = hp[0] + (int32_t)(a.nh * ((int64_t)ez * N));
        const double *cp = a.scol + eh * 13 * PP + c, *lp = a.slay + 4 * ((int64_t)ez * P + k);
        const double ir = lp[0], ihz = lp[1], jwk = lp[2], ga = lp[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            in.mx[d] = (T)(cp[d * PP] * ir);
            in.mx[3 + d] = (T)(cp[(3 + d) * PP] * ir);
            in.mx[6 + d] = (T)(cp[(6 + d) * PP] * ihz);
            in.gv[d] = (T)(-ga * cp[(10 + d) * PP]);
        }
        in.mx[9] = (T)(cp[9 * PP] * jwk);
    } else if constexpr (SHELL) {
        in.I = a.G[e * NP + l];
    } else {
        const BoxElem be = box_elem((uint32_t)e, a.fx, a.fy);
        in.I = box_unique<N, T>(a, be, i, j, k);
        in.ez = be.ez;
        if constexpr (GEO == kMetricBox) {
            const double *cp = a.hcol + (int64_t)(be.ex + a.nx * be.ey) * (4 * PP) + (i + P * j);
            in.c0 = cp[0] * a.w[k];
            in.c1 = cp[PP];
            in.c2 = cp[2 * PP];
            in.c3 = cp[3 * PP];
            in.zk = a.xi[k];
        }
    }
    if constexpr (GEO == kMetricStored) {
        const T *mp = a.met + e * 10 * NP + l;
#pragma unroll
        for (int c = 0; c < 10; ++c) in.mx[c] = mp[c * NP];
    }
    const double *qp = a.q + in.I;
    in.rp = qp[0];
    in.u = qp[a.nu];
    in.v = qp[2 * a.nu];
    in.w = qp[3 * a.nu];
    in.tp = qp[4 * a.nu];
    const double *rf = a.ref + in.I;
    in.rb = rf[0];
    in.tb = rf[a.nu];
    in.pb = rf[2 * a.nu];
}

template <int N, typename T, bool SHELL, int GEO = kMetricStored>
__device__ __forceinline__ void node_stage(const RhsArgs<T> &a, int64_t e, int l, const NodeIn<T> &in,
                                           T (*s)[(N + 1) * (N + 1) * (N + 1)])
{
    constexpr int NP = (N + 1) * (N + 1) * (N + 1);
    if (l >= NP) return;
    const double rho = in.rb + in.rp;
    // p' = p_bar ((rho theta / rho_bar theta_bar)^gamma - 1) without cancellation
    const double dl = in.rp * in.tb + in.rb * in.tp + in.rp * in.tp;
    const double pp = in.pb * eos_rel(dl / (in.rb * in.tb), a.gamma, a.eos);
    s[0][l] = (T)(rho * in.u);
    s[1][l] = (T)(rho * in.v);
    s[2][l] = (T)(rho * in.w);
    s[3][l] = (T)in.u;
    s[4][l] = (T)in.v;
    s[5][l] = (T)in.w;
    s[6][l] = (T)in.tp;
    s[7][l] = (T)pp;
    if constexpr (SHELL) {
        // the background theta is differentiated relative to the element's first node
        const double t0 = a.ref[a.nu + (GEO == kMetricShell ? in.I0 : a.G[e * NP])];
        s[8][l] = (T)(in.tb - t0);
    }
}

// rows i, j, k of D for node l (l < (N+1)^3)
template <int N, typename T>
__device__ __forceinline__ void d_rows(const T *D, int l, T *Di, T *Dj, T *Dk)
{
    constexpr int P = N + 1, PP = P * P;
    const int i = l % P, j = (l / P) % P, k = l / PP;
#pragma unroll
    for (int m = 0; m < P; ++m) {
        Di[m] = D[i * P + m];
        Dj[m] = D[j * P + m];
        Dk[m] = D[k * P + m];
    }
}

// metric of a box node with the recomputed metric: column factors c0..c3,
// element layer ez and xi_k
template <typename T>
__device__ __forceinline__ void box_node_metric(const BoxMetric &bm, int ez, double zk, double c0, double c1, double c2,
                                                double c3, T *mx)
{
    const double omz = 1.0 - ((double)ez + 0.5 * (1.0 + zk)) * bm.inz;  // 1 - z/H
    mx[0] = (T)bm.ixa;
    mx[4] = (T)bm.iyb;
    mx[6] = (T)(omz * c2);
    mx[7] = (T)(omz * c3);
    mx[8] = (T)c1;
    mx[9] = (T)c0;
}

// R at one node from the reference derivatives dd[f][d] of the tile fields
// (d = xi, eta, zeta) and the metric mx: the chain rule, for the advected
// fields directly in contravariant form, u . grad f = sum_d U_d df/dxi_d with
// U_d = u . grad(xi_d).  With GEO == kMetricBox only the entries of the
// box metric are read (xi_x, eta_y, zeta_x, zeta_y, zeta_z), and the
// contractions the chain rule does not use are never formed.
template <typename T, bool SHELL, int GEO>
__device__ __forceinline__ void node_combine(const RhsArgs<T> &a, const T (*dd)[3], const T *mx, double u, double v,
                                             double w, double rp, double rb, const T *gv, NodeOut<T> &o)
{
    const T uu = (T)u, vv = (T)v, ww = (T)w;
    T Uc[3];
    if constexpr (GEO == kMetricBox) {
        Uc[0] = uu * mx[0];
        Uc[1] = vv * mx[4];
        Uc[2] = uu * mx[6] + vv * mx[7] + ww * mx[8];
    } else {
        Uc[0] = uu * mx[0] + vv * mx[1] + ww * mx[2];
        Uc[1] = uu * mx[3] + vv * mx[4] + ww * mx[5];
        Uc[2] = uu * mx[6] + vv * mx[7] + ww * mx[8];
    }
    // Cartesian derivative d/dx_c of field f (row c of the inverse metric)
    auto cart = [&](int f, int c) -> T {
        if constexpr (GEO == kMetricBox) {
            if (c == 0) return dd[f][0] * mx[0] + dd[f][2] * mx[6];
            if (c == 1) return dd[f][1] * mx[4] + dd[f][2] * mx[7];
            return dd[f][2] * mx[8];
        } else {
            return dd[f][0] * mx[c] + dd[f][1] * mx[3 + c] + dd[f][2] * mx[6 + c];
        }
    };
    auto adv = [&](int f) -> T { return Uc[0] * dd[f][0] + Uc[1] * dd[f][1] + Uc[2] * dd[f][2]; };
    const double irho64 = 1.0 / (rb + rp);
    const T irho = (T)irho64;
    const T buoy = (T)(rp * irho64);
    T gx = 0, gy = 0, gz = (T)(-a.g0);
    if constexpr (SHELL) {
        gx = gv[0];
        gy = gv[1];
        gz = gv[2];
    }
    o.R[0] = -(cart(0, 0) + cart(1, 1) + cart(2, 2));
    o.R[1] = -adv(3) - cart(7, 0) * irho + buoy * gx;
    o.R[2] = -adv(4) - cart(7, 1) * irho + buoy * gy;
    o.R[3] = -adv(5) - cart(7, 2) * irho + buoy * gz;
    o.R[4] = -adv(6);
    if constexpr (SHELL) o.R[4] -= adv(8);
    o.Jw = mx[9];
}

template <int N, typename T, bool SHELL, int GEO>
__device__ __forceinline__ void node_derive(const RhsArgs<T> &a, int l, const NodeIn<T> &in, const T *Di,
                                            const T *Dj, const T *Dk, T (*s)[(N + 1) * (N + 1) * (N + 1)],
                                            NodeOut<T> &o)
{
    constexpr int P = N + 1, PP = P * P;
    const int i = l % P, j = (l / P) % P, k = l / PP;
    T mx[10];
    if constexpr (GEO == kMetricBox) {
        box_node_metric<T>(a.bm, in.ez, in.zk, in.c0, in.c1, in.c2, in.c3, mx);
    } else {  // stored, or the shell's recomputed metric (formed by node_gather)
#pragma unroll
        for (int c = 0; c < 10; ++c) mx[c] = in.mx[c];
    }
    // reference derivatives of every field (the unused ones are dropped by
    // the compiler), then R
    constexpr int NF = SHELL ? 9 : 8;
    T dd[NF][3];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        T da = 0, db = 0, dc = 0;
#pragma unroll
        for (int m = 0; m < P; ++m) {
            da += Di[m] * s[f][m + P * (j + P * k)];
            db += Dj[m] * s[f][i + P * (m + P * k)];
            dc += Dk[m] * s[f][i + P * (j + P * m)];
        }
        dd[f][0] = da;
        dd[f][1] = db;
        dd[f][2] = dc;
    }
    T gv[3] = {0, 0, 0};
    if constexpr (SHELL && GEO == kMetricShell) {
        gv[0] = in.gv[0];
        gv[1] = in.gv[1];
        gv[2] = in.gv[2];
    } else if constexpr (SHELL) {
        gv[0] = (T)a.grav[in.I];
        gv[1] = (T)a.grav[a.nu + in.I];
        gv[2] = (T)a.grav[2 * a.nu + in.I];
    }
    node_combine<T, SHELL, GEO>(a, dd, mx, in.u, in.v, in.w, in.rp, in.rb, gv, o);
}

// node_derive for the box's recomputed metric with R accumulated direction
// by direction: every term of R is linear in the reference derivatives, so
// the xi terms of all fields are added first (row i of D), then the eta
// terms (row j), then the zeta terms (row k).  One row of D and five sums
// are live instead of three rows and 24 derivatives (the one-node-per-lane
// kernel at 64x64x16: N = 7 1197 -> 1040 us, N = 8 2491 -> 2467 us; no gain
// on the shell's or the stored metric's kernels, which keep node_derive).
// The same terms as node_combine (GEO == kMetricBox), summed in another
// order.
template <int N, typename T>
__device__ __forceinline__ void node_derive_box_dirs(const RhsArgs<T> &a, int l, const NodeIn<T> &in,
                                                     T (*s)[(N + 1) * (N + 1) * (N + 1)], NodeOut<T> &o)
{
    constexpr int P = N + 1, PP = P * P;
    const int i = l % P, j = (l / P) % P, k = l / PP;
    T mx[10];
    box_node_metric<T>(a.bm, in.ez, in.zk, in.c0, in.c1, in.c2, in.c3, mx);
    const T uu = (T)in.u, vv = (T)in.v, ww = (T)in.w;
    const T Uc0 = uu * mx[0], Uc1 = vv * mx[4], Uc2 = uu * mx[6] + vv * mx[7] + ww * mx[8];
    const double irho64 = 1.0 / (in.rb + in.rp);
    const T irho = (T)irho64;
    // A: the sums whose negatives are R (tile fields: 0 rho u, 1 rho v,
    // 2 rho w, 3 u, 4 v, 5 w, 6 theta', 7 p')
    T A[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int r = d == 0 ? i : (d == 1 ? j : k);
        T Dr[P];
#pragma unroll
        for (int m = 0; m < P; ++m) Dr[m] = a.D[r * P + m];
        auto dfd = [&](int f) -> T {
            T acc = 0;
#pragma unroll
            for (int m = 0; m < P; ++m) {
                const int at = d == 0 ? m + P * (j + P * k) : (d == 1 ? i + P * (m + P * k) : i + P * (j + P * m));
                acc += Dr[m] * s[f][at];
            }
            return acc;
        };
        const T U = d == 0 ? Uc0 : (d == 1 ? Uc1 : Uc2);
        // continuity: d(rho u)/dx = rho u_xi xi_x + rho u_zeta zeta_x, and so on
        if (d == 0) A[0] += dfd(0) * mx[0];
        if (d == 1) A[0] += dfd(1) * mx[4];
        if (d == 2) A[0] += dfd(0) * mx[6] + dfd(1) * mx[7] + dfd(2) * mx[8];
        // advection of u, v, w, theta'
#pragma unroll
        for (int f = 3; f < 7; ++f) A[f - 2] += U * dfd(f);
        // pressure gradient over rho
        const T dp = dfd(7);
        if (d == 0) A[1] += irho * (dp * mx[0]);
        if (d == 1) A[2] += irho * (dp * mx[4]);
        if (d == 2) {
            A[1] += irho * (dp * mx[6]);
            A[2] += irho * (dp * mx[7]);
            A[3] += irho * (dp * mx[8]);
        }
    }
    const T buoy = (T)(in.rp * irho64);
    o.R[0] = -A[0];
    o.R[1] = -A[1];
    o.R[2] = -A[2];
    o.R[3] = -A[3] + buoy * (T)(-a.g0);
    o.R[4] = -A[4];
    o.Jw = mx[9];
}

// Gathers the element tile, differentiates it and evaluates R at node l of
// element e.  Must be called by all lanes of the block (it synchronises);
// returns false for the padding lanes (l >= (N+1)^3).
template <int N, typename T, bool SHELL, int GEO = kMetricStored>
__device__ __forceinline__ bool element_rhs(const RhsArgs<T> &a, int64_t e, int l, T (*s)[(N + 1) * (N + 1) * (N + 1)],
                                            NodeOut<T> &o)
{
    constexpr int P = N + 1, NP = P * P * P;
    NodeIn<T> in;
    node_gather<N, T, SHELL, GEO>(a, e, l, in);
    node_stage<N, T, SHELL, GEO>(a, e, l, in, s);
    __syncthreads();
    if (l >= NP) return false;
    T Di[P], Dj[P], Dk[P];
    d_rows<N, T>(a.D, l, Di, Dj, Dk);
    node_derive<N, T, SHELL, GEO>(a, l, in, Di, Dj, Dk, s, o);
    return true;
}

struct PointArgs {
    const int32_t *off, *idx;
    const double *Minv, *nrm;
    int64_t nl, nu, nh;
    int walls;
};

// The inverse mass that matches the J w of the mesh's element kernels: with
// the recomputed metric they form J w from the column (and layer) factors,
// and the stages, and the box filter, which takes J w the same way, divide by
// the sum of those (MinvR); otherwise by the sum of the stored J w.
inline const double *stage_minv(const Mesh &m)
{
    return m.metric_mode == NUMA_METRIC_RECOMPUTE ? m.dv.MinvR : m.dv.Minv;
}

inline PointArgs point_args(const Mesh &m)
{
    PointArgs p;
    p.off = m.dv.off;
    p.idx = m.dv.idx;
    p.Minv = m.dv.Minv;
    p.nrm = m.dv.nrm;
    p.nl = m.nl;
    p.nu = m.nu;
    p.nh = m.nh;
    p.walls = m.walls ? 1 : 0;
    return p;
}

// remove the wall-normal component of (r1, r2, r3) at bottom/top nodes
__device__ inline void noflux(const PointArgs &p, int64_t I, double &r1, double &r2, double &r3)
{
    if (!p.walls) return;
    int side;
    int64_t h;
    if (I < p.nh) { side = 0; h = I; }
    else if (I >= p.nu - p.nh) { side = 1; h = I - (p.nu - p.nh); }
    else return;
    const double *n = p.nrm + side * 3 * p.nh + h;
    double n0 = n[0], n1 = n[p.nh], n2 = n[2 * p.nh];
    double dn = r1 * n0 + r2 * n1 + r3 * n2;
    r1 -= dn * n0;
    r2 -= dn * n1;
    r3 -= dn * n2;
}

// Sets *flag (when given) if any of the n values is not finite: a plain store
// of 1 by every such lane, the flag is never cleared here.
__device__ __forceinline__ void flag_nonfinite(int32_t *flag, const double *v, int n)
{
    if (!flag) return;
    bool bad = false;
    for (int k = 0; k < n; ++k) bad |= !isfinite(v[k]);
    if (bad) *flag = 1;
}

// Runge-Kutta stage update (Shu-Osher form, StageCoef): y = q_s + cdt R, then
// q_out = a q_ref + b y (y itself when a = 0 and b = 1); with b = 0 the update
// is q_ref a + cdt R (the explicit leap-frog step: q_s is not used).  The
// contractions are written out (fma) so that every kernel that updates a state
// from a summed R rounds it the same way (the box's FP64 stages form q_s +
// cdt R per copy instead: see box_finish_node).
__device__ inline double rk_update(const StageCoef &c, double qref, double qs, double r)
{
    if (c.b == 0.0) return fma(c.cdt, r, c.a * qref);
    const double y = fma(c.cdt, r, qs);
    if (c.a == 0.0 && c.b == 1.0) return y;
    return fma(c.b, y, c.a * qref);
}

// The same update when the element kernel has already formed y = q_s + cdt R
// inside its contributions (b != 0; see box_finish_node's fold).
__device__ inline double rk_update_folded(const StageCoef &c, double qref, double y)
{
    if (c.a == 0.0 && c.b == 1.0) return y;
    return fma(c.b, y, c.a * qref);
}

// Finish of a fused stage on the box.  A block takes SEG consecutive elements
// along x of one (ey, ez) (sx: the segment index along x) and, per element,
// the lattice nodes whose lower corner it is (local 0 <= i, j, k < N); lanes
// run along x fastest, so every state read and write covers SEG*N consecutive
// unique ids.  The copies of a node follow from its lattice position: on an
// element face along a direction it has two copies (local index 0 of the
// element above and N of the one below, wrapped when periodic), else one.  A
// second launch with kbase = N, klayers = 1 covers the top wall layer
// (ez = nz - 1).  Indices are 32-bit: the mesh keeps n_local, n_unique < 2^31.
// PLAIN: the output is the summed, mass-weighted and projected value itself
// (the filter's DSS); qs and qn are not read.
// fold: away from the walls the contributions are J w (q_s + cdt R) (the
// element kernel has the stage state of its nodes at hand), so their mass-
// weighted sum is y = q_s + cdt R itself, since the mass is the sum of the
// copies' J w, and q_s is not read there; wall nodes carry J w R, as the
// no-flux projection acts on R alone.  The mass must then sum the same J w
// as the contributions: with the recomputed metric p.Minv is MinvR (the
// stored isoparametric J w differs from c0 w_k by ~1e-14, which the fold
// would apply to the state at every stage).
struct BoxFin {
    int nx, ny, nz, walls;
    int ni, nj;
    int fold;
};

template <int N, int SEG, typename T, bool PLAIN = false>
__device__ __forceinline__ void box_finish_node(const PointArgs &p, const BoxFin &b, const T *ev, int sx, int ey,
                                                int ez, int lane, int kbase, int klayers, const StageCoef &sc,
                                                const double *qn, const double *qs, double *qout,
                                                int32_t *flag = nullptr)
{
    constexpr int P = N + 1, NP = P * P * P, W = SEG * N;
    if (lane >= W * N * klayers) return;
    const int a = lane % W, jj = (lane / W) % N, kk = lane / (W * N);
    const int gi = sx * W + a, gj = ey * N + jj, gk = ez * N + kbase + kk;
    const int32_t I = gi + b.ni * (gj + b.nj * gk);
    // copies along each direction: (element index along the direction, local index)
    int cx[2], cy[2], cz[2];
    int lx[2], ly[2], lz[2], nxc, nyc, nzc;
    const int exa = sx * SEG + a / N;
    if (a % N == 0) {  // gi is a multiple of N: element face in x
        cx[0] = exa; lx[0] = 0;
        cx[1] = exa == 0 ? b.nx - 1 : exa - 1; lx[1] = N;
        nxc = 2;
    } else {
        cx[0] = exa; lx[0] = a % N;
        nxc = 1;
    }
    if (jj == 0) {
        cy[0] = ey; ly[0] = 0;
        cy[1] = ey == 0 ? b.ny - 1 : ey - 1; ly[1] = N;
        nyc = 2;
    } else {
        cy[0] = ey; ly[0] = jj;
        nyc = 1;
    }
    const int kl = kbase + kk;  // local k in element ez
    if (kl == 0) {
        if (ez == 0 && b.walls) {
            cz[0] = 0; lz[0] = 0; nzc = 1;
        } else {
            cz[0] = ez; lz[0] = 0;
            cz[1] = ez == 0 ? b.nz - 1 : ez - 1; lz[1] = N;
            nzc = 2;
        }
    } else {
        cz[0] = ez; lz[0] = kl; nzc = 1;  // kl == N only for the top wall layer
    }
    // the loads that do not depend on the sum are issued first
    const double *qsi = qs + I, *qni = qn + I;
    double *qoi = qout + I;
    const double mi = p.Minv[I];
    const bool wall = b.walls && ((ez == 0 && kl == 0) || kl == N);
    const bool folded = !PLAIN && b.fold && !wall;
    double qsv[5] = {0, 0, 0, 0, 0}, qnv[5] = {0, 0, 0, 0, 0};
    if (!PLAIN)
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            qsv[v] = folded ? 0.0 : qsi[v * p.nu];
            qnv[v] = sc.a == 0.0 ? 0.0 : qni[v * p.nu];
        }
    // copies of one z layer: the up to four (y, x) copies are loaded together
    // (absent ones are not loaded and count zero), so a node waits for one
    // round trip per z layer instead of one per copy
    if (nxc == 1) { cx[1] = cx[0]; lx[1] = lx[0]; }
    if (nyc == 1) { cy[1] = cy[0]; ly[1] = ly[0]; }
    double r[5] = {0, 0, 0, 0, 0};
    for (int z = 0; z < nzc; ++z) {
        T c[4][5];
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                const int32_t e = cx[x] + b.nx * (cy[y] + b.ny * cz[z]);
                const int32_t cc = e * NP + lx[x] + P * (ly[y] + P * lz[z]);
                const T *src = ev + (int64_t)cc * 5;  // node-major [n_local][5]
                if (y < nyc && x < nxc) {
#pragma unroll
                    for (int v = 0; v < 5; ++v) c[2 * y + x][v] = src[v];
                } else {
#pragma unroll
                    for (int v = 0; v < 5; ++v) c[2 * y + x][v] = (T)0;
                }
            }
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                const bool has = y < nyc && x < nxc;
#pragma unroll
                for (int v = 0; v < 5; ++v) r[v] += has ? (double)c[2 * y + x][v] : 0.0;
            }
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) r[v] *= mi;
    double o[5];
    if (folded) {
#pragma unroll
        for (int v = 0; v < 5; ++v) o[v] = rk_update_folded(sc, qnv[v], r[v]);
    } else {
        noflux(p, I, r[1], r[2], r[3]);
#pragma unroll
        for (int v = 0; v < 5; ++v) o[v] = PLAIN ? r[v] : rk_update(sc, qnv[v], qsv[v], r[v]);
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) qoi[v * p.nu] = o[v];
    flag_nonfinite(flag, o, 5);
}

// Copy n values staged in LDS (st) to out with 16-byte stores: the leading values until out is 16-byte aligned one by one, then
// 16-byte vectors (two FP64 or four FP32 values per lane), then the tail.
template <typename T>
__device__ __forceinline__ void store_run(T *out, const T *st, int n, int t, int nthreads)
{
    using V = typename std::conditional<sizeof(T) == 8, double2, float4>::type;
    constexpr int W = 16 / sizeof(T);
    int lead = (int)(((16 - ((uintptr_t)out & 15)) & 15) / sizeof(T));
    if (lead > n) lead = n;
    if (t < lead) out[t] = st[t];
    const int nv = (n - lead) / W;
    const T *sv = st + lead;
    V *ov = reinterpret_cast<V *>(out + lead);
    for (int u = t; u < nv; u += nthreads) {
        V val;
        T *vp = reinterpret_cast<T *>(&val);
#pragma unroll
        for (int c = 0; c < W; ++c) vp[c] = sv[u * W + c];
        ov[u] = val;
    }
    for (int u = lead + nv * W + t; u < n; u += nthreads) out[u] = st[u];
}

// x-segment length of a box finish block: whole 128-byte lines of FP64 state
// where the block fits in 1024 lanes
template <int N>
constexpr int seg_for() { return 4 * N * N * N <= 1024 ? 4 : (2 * N * N * N <= 1024 ? 2 : 1); }

}  // namespace dev
}  // namespace numa
