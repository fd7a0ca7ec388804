// 1D-IMEX vertical correction (Sec. "Time Discretization": implicit
// corrections along the vertical columns after an explicit leap-frog step;
// Code example 1: "compute IMEX corrections for each vertical column").
//
// After the explicit leap-frog step q* = q^{n-1} + 2 dt L(q^n) (a fused stage
// with the update a q_ref + cdt R), the linearised vertical terms V are taken
// as the trapezoidal mean of the new and the old level:
//   (I - dt V) q^{n+1} = q* - dt V(2 q^n - q^{n-1}),
// then the Robert-Asselin filter q^n <- q^n + ra (q^{n-1} - 2 q^n + q^{n+1}).
// With n the unit vertical (z on the box, radial on the shell), w = u.n and
// s = 1 (box) or r^2 (shell), V linearised about the hydrostatic reference is
//   V_rho' = -(1/s) G(s rho_bar w),
//   V_w    = -(1/rho_bar) G(c2 rho' + kap theta') + g_n rho'/rho_bar   (along n),
//   V_theta' = -beta w,  beta = G(theta_bar),
// with c2 = gamma p_bar / rho_bar, kap = c2 rho_bar / theta_bar, g_n = g.n, and
// zero momentum rows at the walls.  d/dn acts along zeta only in both maps, and
// the DSS of an element-local zeta derivative reduces on a vertical lattice
// line to the 1D operator
//   (G f)_g = sum_{e ∋ g} w_k(g) (D f_e)_k(g) / sum_{e ∋ g} h_e(g) w_k(g),
// h_e = dn/dzeta of element e at the node (z_zeta, or the shell's radial
// h_zeta): the horizontal copies of a node contribute identical terms, and
// on the shell r^2 cancels between J w and the mass.  So each line is an
// independent system in (rho', w, theta'); eliminating
// rho' = r_rho - (dt/s) G(s rho_bar w) and theta' = r_theta - dt beta w leaves
//   A w = r_w - dt (1/rho_bar) G(c2 r_rho + kap r_theta) + dt (g_n/rho_bar) r_rho,
//   A = I - dt^2 (1/rho_bar) G c2 s^-1 G s rho_bar - dt^2 (1/rho_bar) G kap beta
//         + dt^2 (g_n / rho_bar) s^-1 G s rho_bar
// (wall rows: w = r_w), a band matrix of half-width 2N that depends on dt and
// the reference state only.  It is factored once per dt (LU without pivoting:
// I plus dt^2 times a vertical acoustic operator) into the workspace; every
// step then streams each line bottom to top and back, one lane per line, so
// that neighbouring lanes read neighbouring lattice lines (coalesced).  The
// new velocity is the explicit one with its n component replaced.
#include "kernels.h"

namespace numa {
namespace {

struct ImexArgs {
    const double *qs;      // q*: the explicit leap-frog step, [5][n_unique]
    double *qcur, *qprev;  // in: q^n, q^{n-1}; out: q^{n+1}, the filtered q^n
    const double *ref;     // [3][n_unique]: rho_bar, theta_bar, p_bar
    const double *hcol;    // box column factors, 1/z_zeta in factor 1
    const double *slay;    // shell layer factors [nz (N+1)][4]: 1/r, 1/h_zeta, ., g0 (a/r)^2
    const double *xu;      // [3][n_unique] coordinates (the shell's radial direction)
    double *lu;            // [n_levels][4N+1][n_lines]: L below, 1/U_gg on, U above the diagonal
    double *sr, *sx, *st, *sb;  // [n_levels][n_lines] line vectors: r_rho; r_w, y, w; r_theta; beta
    int64_t nu, nh;        // unique nodes, lines (horizontal unique nodes)
    int ni, nk, nx, shell; // box: lattice extent along x, elements along x; levels
    double dt, ra, gamma, gz, theta0;
    double D[kMaxP * kMaxP], w[kMaxP];
};

// Per-line geometry: the box's z_zeta is the same for the whole line; the
// shell's radial factors come per (layer, local k).
struct LineGeo {
    double izz;     // box: 1/z_zeta
    double n[3];    // unit vertical
};

template <int N>
__device__ __forceinline__ LineGeo line_geo(const ImexArgs &a, int64_t L)
{
    constexpr int P = N + 1, PP = P * P;
    LineGeo lg;
    if (a.shell) {
        const double x = a.xu[L], y = a.xu[a.nu + L], z = a.xu[2 * a.nu + L];
        const double ir = 1.0 / sqrt(x * x + y * y + z * z);
        lg.n[0] = x * ir;
        lg.n[1] = y * ir;
        lg.n[2] = z * ir;
        lg.izz = 0.0;
    } else {
        const int gi = (int)(L % a.ni), gj = (int)(L / a.ni);
        const int ex = gi / N, ey = gj / N;
        lg.izz = a.hcol[(int64_t)(ex + a.nx * ey) * (4 * PP) + PP + (gi - ex * N) + P * (gj - ey * N)];
        lg.n[0] = 0.0;
        lg.n[1] = 0.0;
        lg.n[2] = 1.0;
    }
    return lg;
}

// dn/dzeta of element e at its local node k
template <int N>
__device__ __forceinline__ double h_of(const ImexArgs &a, const LineGeo &lg, int e, int k)
{
    return a.shell ? 1.0 / a.slay[4 * (e * (N + 1) + k) + 1] : 1.0 / lg.izz;
}

// s (r^2 on the shell) and g.n at level g of the line
template <int N>
__device__ __forceinline__ void level_factors(const ImexArgs &a, int g, double &s, double &gn)
{
    if (a.shell) {
        int e = g / N, k = g - e * N;
        if (e >= (a.nk - 1) / N) {  // the top node: element below, local N
            e -= 1;
            k = N;
        }
        const double ir = a.slay[4 * (e * (N + 1) + k)];
        s = 1.0 / (ir * ir);
        gn = -a.slay[4 * (e * (N + 1) + k) + 3];
    } else {
        s = 1.0;
        gn = a.gz;
    }
}

// (G)_{g m} on a line of nk = nz N + 1 levels
template <int N>
__device__ double g_entry(const ImexArgs &a, const LineGeo &lg, int g, int m)
{
    constexpr int P = N + 1;
    double num = 0.0, den = 0.0;
    const int eg = g / N, kg = g - eg * N;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        // element eg (local kg) and, on an element boundary, eg - 1 (local N)
        const int e = s == 0 ? eg : eg - 1, k = s == 0 ? kg : N;
        if (s == 0 && g == a.nk - 1) continue;  // top wall node: element below only
        if (s == 1 && (kg != 0 || eg == 0)) continue;
        den += h_of<N>(a, lg, e, k) * a.w[k];
        const int km = m - e * N;
        if (km >= 0 && km <= N) num += a.w[k] * a.D[k * P + km];
    }
    return num / den;
}

// The factors of A for every line: one 64-lane workgroup per line builds the
// band of G and of A in LDS, factors it and writes the band out.
template <int N>
__global__ __launch_bounds__(64) void k_imex_factor(ImexArgs a)
{
    constexpr int B = 2 * N, W = 2 * B + 1, GW = 2 * N + 1;
    extern __shared__ double sm[];
    const int nk = a.nk, lane = threadIdx.x;
    double *Ab = sm;               // [nk][W]: A_{g m} at g W + m - g + B
    double *Gb = Ab + nk * W;      // [nk][GW]: G_{g m} at g GW + m - g + N
    double *rb = Gb + nk * GW, *c2 = rb + nk, *sv = c2 + nk, *gn = sv + nk, *kb = gn + nk, *tb = kb + nk;
    const int64_t L = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t nh = a.nh;
    const LineGeo lg = line_geo<N>(a, L);
    for (int g = lane; g < nk; g += 64) {
        const int64_t I = L + nh * g;
        rb[g] = a.ref[I];
        c2[g] = a.gamma * a.ref[2 * a.nu + I] / a.ref[I];
        tb[g] = a.shell ? a.ref[a.nu + I] : a.theta0;
        level_factors<N>(a, g, sv[g], gn[g]);
    }
    for (int t = lane; t < nk * GW; t += 64) {
        const int g = t / GW, m = g + t % GW - N;
        Gb[t] = (m >= 0 && m < nk) ? g_entry<N>(a, lg, g, m) : 0.0;
    }
    __syncthreads();
    // kap beta at every level, beta = G(theta_bar)
    for (int g = lane; g < nk; g += 64) {
        double beta = 0.0;
        for (int d = 0; d < GW; ++d) {
            const int m = g + d - N;
            if (m >= 0 && m < nk) beta += Gb[g * GW + d] * tb[m];
        }
        kb[g] = a.shell ? c2[g] * rb[g] / tb[g] * beta : 0.0;  // theta_bar is constant on the box
    }
    __syncthreads();
    const double dt2 = a.dt * a.dt;
    for (int t = lane; t < nk * W; t += 64) {
        const int g = t / W, m = g + t % W - B;
        double v = 0.0;
        if (m >= 0 && m < nk) {
            if (g == 0 || g == nk - 1) {
                v = m == g ? 1.0 : 0.0;
            } else {
                double acc = 0.0;  // (G c2 s^-1 G)_{g m}
                const int p0 = (g > m ? g : m) - N, p1 = (g < m ? g : m) + N;
                for (int p = p0 < 0 ? 0 : p0; p <= p1 && p < nk; ++p)
                    acc += Gb[g * GW + p - g + N] * (c2[p] / sv[p]) * Gb[p * GW + m - p + N];
                const double gm = (m - g >= -N && m - g <= N) ? Gb[g * GW + m - g + N] : 0.0;
                v = (m == g ? 1.0 : 0.0) - dt2 / rb[g] * acc * sv[m] * rb[m] - dt2 / rb[g] * gm * kb[m] +
                    dt2 * gn[g] / (rb[g] * sv[g]) * gm * sv[m] * rb[m];
            }
        }
        Ab[t] = v;
    }
    __syncthreads();
    // band LU without pivoting; multipliers below the diagonal
    for (int k = 0; k < nk - 1; ++k) {
        const int rmax = k + B < nk - 1 ? k + B : nk - 1;
        if (lane < B && k + 1 + lane <= rmax) {
            const int r = k + 1 + lane;
            Ab[r * W + k - r + B] /= Ab[k * W + B];
        }
        __syncthreads();
        for (int t = lane; t < B * B; t += 64) {
            const int r = k + 1 + t / B, c = k + 1 + t % B;
            if (r <= rmax && c <= rmax) Ab[r * W + c - r + B] -= Ab[r * W + k - r + B] * Ab[k * W + c - k + B];
        }
        __syncthreads();
    }
    // out, [g][d][line]; entries outside the line are zero, the diagonal is
    // stored as its reciprocal
    for (int t = lane; t < nk * W; t += 64) a.lu[(int64_t)t * nh + L] = t % W == B ? 1.0 / Ab[t] : Ab[t];
}

// D f on one element's nodes (the zeta derivative); D from LDS (uniform
// addresses: one broadcast read per entry)
template <int N>
__device__ __forceinline__ void dloc(const double *D, const double (&f)[N + 1], double (&df)[N + 1])
{
    constexpr int P = N + 1;
    // read D where it is used: kept live across the element loop it would
    // take (N+1)^2 register pairs
    asm volatile("" ::: "memory");
#pragma unroll
    for (int k = 0; k < P; ++k) {
        double s = 0.0;
#pragma unroll
        for (int m = 0; m < P; ++m) s = fma(D[k * P + m], f[m], s);
        df[k] = s;
    }
}

// G f at local node k of element e: k = 0 above the bottom combines the
// element below through its top derivative dprev and dn/dzeta hprev (the DSS
// of the two copies)
__device__ __forceinline__ double gat(double w0, double wN, int e, int k, double dk, double hk, double dprev,
                                      double hprev)
{
    if (k == 0 && e > 0) return (wN * dprev + w0 * dk) / (wN * hprev + w0 * hk);
    return dk / hk;
}

// One step's vertical correction: one lane per line, four passes along it;
// an element's N+1 nodes at a time, node e N + N finishing with element e + 1
// (or as the top wall node).
template <int N, bool SHELL>
__global__ __launch_bounds__(256) void k_imex_solve(ImexArgs a)
{
    constexpr int P = N + 1, B = 2 * N, W = 2 * B + 1;
    __shared__ double D[P * P];
    if (threadIdx.x < P * P) D[threadIdx.x] = a.D[threadIdx.x];
    __syncthreads();
    const int64_t nh = a.nh, nu = a.nu;
    const int64_t L = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (L >= nh) return;
    const int nk = a.nk, nz = (nk - 1) / N;
    const LineGeo lg = line_geo<N>(a, L);
    // the box's vertical is z, its theta_bar constant (beta = 0)
    const double n0 = SHELL ? lg.n[0] : 0.0, n1 = SHELL ? lg.n[1] : 0.0, n2 = SHELL ? lg.n[2] : 1.0;
    const double dt = a.dt, w0 = a.w[0], wN = a.w[N];
    // pass 1: sigma = 2 q^n - q^{n-1};
    //   r_rho = q*_rho + (dt/s) G(s rho_bar sigma_w), beta = G(theta_bar),
    //   r_w = q*_w + dt (G(c2 sigma_rho + kap sigma_theta) - g_n sigma_rho)/rho_bar (q*_w at walls),
    //   r_theta = q*_theta + dt beta sigma_w
    double cf = 0.0, ch = 0.0, ct = 0.0, hp = 0.0;
    for (int e = 0; e < nz; ++e) {
        double f[P], h[P], tb[P], s0v[P], swv[P], rbv[P], df[P], dh[P], dtb[P], hv[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const int64_t I = L + nh * (e * N + k);
            double s, gn;
            level_factors<N>(a, e * N + k, s, gn);
            const double rbar = a.ref[I], cc = a.gamma * a.ref[2 * nu + I] / rbar;
            const double tbar = a.shell ? a.ref[nu + I] : a.theta0;
            const double s0 = 2.0 * a.qcur[I] - a.qprev[I];
            const double sw = SHELL ? n0 * (2.0 * a.qcur[nu + I] - a.qprev[nu + I]) +
                                          n1 * (2.0 * a.qcur[2 * nu + I] - a.qprev[2 * nu + I]) +
                                          n2 * (2.0 * a.qcur[3 * nu + I] - a.qprev[3 * nu + I])
                                    : 2.0 * a.qcur[3 * nu + I] - a.qprev[3 * nu + I];
            const double s4 = 2.0 * a.qcur[4 * nu + I] - a.qprev[4 * nu + I];
            f[k] = s * rbar * sw;
            h[k] = cc * s0 + cc * rbar / tbar * s4;
            tb[k] = tbar;
            s0v[k] = s0;
            swv[k] = sw;
            rbv[k] = rbar;
            hv[k] = h_of<N>(a, lg, e, k);
        }
        dloc<N>(D, f, df);
        dloc<N>(D, h, dh);
        if (SHELL) dloc<N>(D, tb, dtb);
#pragma unroll
        for (int k = 0; k < P; ++k) {
            if (k == N && e != nz - 1) continue;
            const int g = e * N + k;
            const int64_t I = L + nh * g;
            double s, gn;
            level_factors<N>(a, g, s, gn);
            const double gf = gat(w0, wN, e, k, df[k], hv[k], cf, hp);
            const double gh = gat(w0, wN, e, k, dh[k], hv[k], ch, hp);
            const bool wall = g == 0 || g == nk - 1;
            const double qw = SHELL ? n0 * a.qs[nu + I] + n1 * a.qs[2 * nu + I] + n2 * a.qs[3 * nu + I]
                                    : a.qs[3 * nu + I];
            a.sr[g * nh + L] = a.qs[I] + dt * gf / s;
            a.sx[g * nh + L] = wall ? qw : qw + dt * (gh - gn * s0v[k]) / rbv[k];
            if (SHELL) {
                const double beta = gat(w0, wN, e, k, dtb[k], hv[k], ct, hp);
                a.st[g * nh + L] = a.qs[4 * nu + I] + dt * beta * swv[k];
                a.sb[g * nh + L] = beta;
            }
        }
        cf = df[N];
        ch = dh[N];
        ct = SHELL ? dtb[N] : 0.0;
        hp = hv[N];
    }
    // pass 2: right side of the w system, and the forward elimination with L
    double yh[B];  // the last B values, newest first
#pragma unroll
    for (int s = 0; s < B; ++s) yh[s] = 0.0;
    ch = 0.0;
    hp = 0.0;
    for (int e = 0; e < nz; ++e) {
        double h[P], rr[P], rbv[P], dh[P], hv[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const int g = e * N + k;
            const int64_t I = L + nh * g;
            const double rbar = a.ref[I], cc = a.gamma * a.ref[2 * nu + I] / rbar;
            const double tbar = a.shell ? a.ref[nu + I] : a.theta0;
            rr[k] = a.sr[g * nh + L];
            h[k] = cc * rr[k] + cc * rbar / tbar * (SHELL ? a.st[g * nh + L] : a.qs[4 * nu + I]);
            rbv[k] = rbar;
            hv[k] = h_of<N>(a, lg, e, k);
        }
        dloc<N>(D, h, dh);
#pragma unroll
        for (int k = 0; k < P; ++k) {
            if (k == N && e != nz - 1) continue;
            const int g = e * N + k;
            double s, gn;
            level_factors<N>(a, g, s, gn);
            const double gh = gat(w0, wN, e, k, dh[k], hv[k], ch, hp);
            const bool wall = g == 0 || g == nk - 1;
            const double rw = a.sx[g * nh + L];
            double y = wall ? rw : rw - dt * gh / rbv[k] + dt * gn * rr[k] / rbv[k];
            const double *lgp = a.lu + (int64_t)g * W * nh + L;
#pragma unroll
            for (int s = 1; s <= B; ++s) y -= lgp[(B - s) * nh] * yh[s - 1];
#pragma unroll
            for (int s = B - 1; s > 0; --s) yh[s] = yh[s - 1];
            yh[0] = y;
            a.sx[g * nh + L] = y;
        }
        ch = dh[N];
        hp = hv[N];
    }
    // pass 3: back substitution with U, top to bottom
#pragma unroll
    for (int s = 0; s < B; ++s) yh[s] = 0.0;
    for (int g = nk - 1; g >= 0; --g) {
        const double *ug = a.lu + (int64_t)g * W * nh + L;
        double w = a.sx[g * nh + L];
#pragma unroll
        for (int s = 1; s <= B; ++s) w -= ug[(B + s) * nh] * yh[s - 1];
        w *= ug[B * nh];
#pragma unroll
        for (int s = B - 1; s > 0; --s) yh[s] = yh[s - 1];
        yh[0] = w;
        a.sx[g * nh + L] = w;
    }
    // pass 4: rho' = r_rho - (dt/s) G(s rho_bar w), theta' = r_theta - dt beta w,
    // the velocity's n component replaced by w; the Robert-Asselin filter of q^n
    cf = 0.0;
    hp = 0.0;
    for (int e = 0; e < nz; ++e) {
        double f[P], wv[P], df[P], hv[P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const int g = e * N + k;
            const int64_t I = L + nh * g;
            double s, gn;
            level_factors<N>(a, g, s, gn);
            wv[k] = a.sx[g * nh + L];
            f[k] = s * a.ref[I] * wv[k];
            hv[k] = h_of<N>(a, lg, e, k);
        }
        dloc<N>(D, f, df);
#pragma unroll
        for (int k = 0; k < P; ++k) {
            if (k == N && e != nz - 1) continue;
            const int g = e * N + k;
            const int64_t I = L + nh * g;
            double s, gn;
            level_factors<N>(a, g, s, gn);
            const double gf = gat(w0, wN, e, k, df[k], hv[k], cf, hp);
            const double u0 = a.qs[nu + I], u1 = a.qs[2 * nu + I], u2 = a.qs[3 * nu + I], w = wv[k];
            double nv[5];
            nv[0] = a.sr[g * nh + L] - dt * gf / s;
            if (SHELL) {
                const double qw = n0 * u0 + n1 * u1 + n2 * u2;
                nv[1] = u0 - qw * n0 + w * n0;
                nv[2] = u1 - qw * n1 + w * n1;
                nv[3] = u2 - qw * n2 + w * n2;
                nv[4] = a.st[g * nh + L] - dt * a.sb[g * nh + L] * w;
            } else {
                nv[1] = u0;
                nv[2] = u1;
                nv[3] = w;
                nv[4] = a.qs[4 * nu + I];
            }
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                const double vc = a.qcur[v * nu + I], vp = a.qprev[v * nu + I];
                a.qprev[v * nu + I] = vc + a.ra * (vp - 2.0 * vc + nv[v]);
                a.qcur[v * nu + I] = nv[v];
            }
        }
        cf = df[N];
        hp = hv[N];
    }
}

ImexArgs imex_args(Mesh &m, double dt, double ra, double *qprev, double *qcur)
{
    ImexArgs a{};
    a.qs = m.dv.qs;
    a.qcur = qcur;
    a.qprev = qprev;
    a.ref = m.dv.ref;
    a.hcol = m.dv.hcol;
    a.slay = m.dv.slay;
    a.xu = m.dv.xu;
    a.lu = m.dv.imexLU;
    a.sr = m.dv.qs2;
    a.sx = m.dv.qs2 + m.nu;
    a.st = m.dv.qs2 + 2 * m.nu;
    a.sb = m.dv.qs2 + 3 * m.nu;
    a.nu = m.nu;
    a.nh = m.nh;
    a.ni = (int)m.ni;
    a.nk = (int)m.nk;
    a.nx = m.d.ne[0];
    a.shell = m.d.kind == NUMA_MESH_SHELL ? 1 : 0;
    a.dt = dt;
    a.ra = ra;
    a.gamma = m.gamma;
    a.gz = -m.ph.g0;
    a.theta0 = m.ph.T0;
    for (int k = 0; k < m.P * m.P; ++k) a.D[k] = m.D[k];
    for (int k = 0; k < m.P; ++k) a.w[k] = m.w[k];
    return a;
}

template <int N>
int32_t launch_imex_n(const ImexArgs &a, bool factor, size_t lds, hipStream_t s)
{
    if (factor)
        hipLaunchKernelGGL((k_imex_factor<N>), dim3((unsigned)a.nh), dim3(64), lds, s, a);
    else if (a.shell)
        hipLaunchKernelGGL((k_imex_solve<N, true>), dim3((unsigned)((a.nh + 255) / 256)), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_imex_solve<N, false>), dim3((unsigned)((a.nh + 255) / 256)), dim3(256), 0, s, a);
    NUMA_HIP(hipGetLastError());
    return NUMA_OK;
}

int32_t launch_imex(Mesh &m, bool factor, double dt, double ra, double *qprev, double *qcur, hipStream_t s)
{
    const ImexArgs a = imex_args(m, dt, ra, qprev, qcur);
    const size_t lds = (size_t)imex_lds_bytes(m);
    switch (m.N) {
    case 1: return launch_imex_n<1>(a, factor, lds, s);
    case 2: return launch_imex_n<2>(a, factor, lds, s);
    case 3: return launch_imex_n<3>(a, factor, lds, s);
    case 4: return launch_imex_n<4>(a, factor, lds, s);
    case 5: return launch_imex_n<5>(a, factor, lds, s);
    case 6: return launch_imex_n<6>(a, factor, lds, s);
    case 7: return launch_imex_n<7>(a, factor, lds, s);
    default: return launch_imex_n<8>(a, factor, lds, s);
    }
}

}  // namespace

uint64_t imex_lds_bytes(const Mesh &m)
{
    return 8ull * (uint64_t)m.nk * ((4 * m.N + 1) + (2 * m.N + 1) + 6);
}

uint64_t imex_factor_bytes(const Mesh &m)
{
    return 8ull * (uint64_t)m.nk * (4 * m.N + 1) * (uint64_t)m.nh;
}

int32_t launch_imex_factor(Mesh &m, double dt, hipStream_t s)
{
    return launch_imex(m, true, dt, 0.0, nullptr, nullptr, s);
}

int32_t launch_imex_correction(Mesh &m, double dt, double ra, double *qprev, double *qcur, hipStream_t s)
{
    return launch_imex(m, false, dt, ra, qprev, qcur, s);
}

}  // namespace numa
