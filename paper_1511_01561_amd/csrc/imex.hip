// 1D-IMEX vertical correction (Sec. "Time Discretization": implicit
// corrections along the vertical columns after an explicit leap-frog step;
// Code example 1: "compute IMEX corrections for each vertical column").
//
// After the explicit leap-frog step q* = q^{n-1} + 2 dt L(q^n) (a fused stage
// with the update a q_ref + cdt R), the linearised vertical terms V are taken
// as the trapezoidal mean of the new and the old level:
//   (I - dt V) q^{n+1} = q* - dt V(2 q^n - q^{n-1}),
// then the Robert-Asselin filter q^n <- q^n + ra (q^{n-1} - 2 q^n + q^{n+1}).
// V, linearised about the hydrostatic reference, is
//   V_rho' = -G(rho_bar w),  V_w = -(1/rho_bar) G(c2 rho' + kap theta') + g_z rho'/rho_bar,
//   V_theta' = 0 (theta_bar is constant on the box), V_u = V_v = 0,
// with c2 = gamma p_bar / rho_bar, kap = c2 rho_bar / theta0, and zero momentum
// rows at the walls.  In the terrain-following box map d/dz acts along zeta
// only, and the DSS of an element-local zeta derivative reduces on a vertical
// lattice line to the 1D operator
//   (G f)_g = sum_{e ∋ g} w_k(g) (D f_e)_k(g) / (z_zeta sum_{e ∋ g} w_k(g))
// (the horizontal copies of a node contribute identical terms).  So each line
// is an independent system in (rho', w, theta'): theta' = r_theta, and
// eliminating rho' = r_rho - dt G(rho_bar w) leaves for w
//   [I - dt^2 (1/rho_bar) G c2 G rho_bar + dt^2 (g_z/rho_bar) G rho_bar] w
//       = r_w - dt (1/rho_bar) G(c2 r_rho + kap r_theta) + dt (g_z/rho_bar) r_rho
// (wall rows: w = r_w), a band matrix of half-width 2N, factored without
// pivoting (I plus dt^2 times a vertical acoustic operator).
//
// One 64-lane workgroup per vertical line; the band matrix, the band of G and
// the line's vectors live in LDS (dynamic size, nk levels).
#include "kernels.h"

namespace numa {
namespace {

struct ImexArgs {
    const double *qs;      // q*: the explicit leap-frog step, [5][n_unique]
    double *qcur, *qprev;  // in: q^n, q^{n-1}; out: q^{n+1}, the filtered q^n
    const double *ref;     // [3][n_unique]: rho_bar, theta_bar, p_bar
    const double *hcol;    // box column factors, 1/z_zeta in factor 1
    int64_t nu;
    int ni, nj, nk, nx;    // lattice extents, elements along x
    double dt, ra, gamma, gz, theta0;
    double D[kMaxP * kMaxP], w[kMaxP];
};

// (G)_{g m} on a line of nk = nz N + 1 levels, z_zeta^-1 = izz
template <int N>
__device__ double g_entry(const ImexArgs &a, int g, int m, double izz)
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
        den += a.w[k];
        const int km = m - e * N;
        if (km >= 0 && km <= N) num += a.w[k] * a.D[k * P + km];
    }
    return num / den * izz;
}

template <int N>
__global__ __launch_bounds__(64) void k_imex_line(ImexArgs a)
{
    constexpr int B = 2 * N, W = 2 * B + 1, GW = 2 * N + 1, P = N + 1, PP = P * P;
    extern __shared__ double sm[];
    const int nk = a.nk, lane = threadIdx.x;
    double *Ab = sm;               // [nk][W]: A_{g m} at g W + m - g + B
    double *Gb = Ab + nk * W;      // [nk][GW]: G_{g m} at g GW + m - g + N
    double *rb = Gb + nk * GW, *c2 = rb + nk, *kap = c2 + nk;
    double *rr = kap + nk, *rw = rr + nk, *rt = rw + nk;  // r = q* - dt V(2 q^n - q^{n-1})
    double *f = rt + nk, *h = f + nk, *x = h + nk;
    double *qc = x + nk, *qp = qc + 3 * nk;  // [3][nk] q^n, q^{n-1} of rho', w, theta'
    const int64_t L = xcd_remap(blockIdx.x, gridDim.x);
    const int gi = (int)(L % a.ni), gj = (int)(L / a.ni);
    const int64_t nh = (int64_t)a.ni * a.nj, nu = a.nu;
    const int ex = gi / N, ey = gj / N;
    const double izz = a.hcol[(int64_t)(ex + a.nx * ey) * (4 * PP) + PP + (gi - ex * N) + P * (gj - ey * N)];
    const double dt = a.dt;
    // line data; u and v are final here (no vertical terms): q^{n+1} = q*
    for (int g = lane; g < nk; g += 64) {
        const int64_t I = L + nh * g;
        const double rbar = a.ref[I], pbar = a.ref[2 * nu + I];
        const double cc = a.gamma * pbar / rbar;
        rb[g] = rbar;
        c2[g] = cc;
        kap[g] = cc * rbar / a.theta0;
        const int cv[3] = {0, 3, 4};
        double s[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double vc = a.qcur[cv[c] * nu + I], vp = a.qprev[cv[c] * nu + I];
            qc[c * nk + g] = vc;
            qp[c * nk + g] = vp;
            s[c] = 2.0 * vc - vp;
        }
        f[g] = rbar * s[1];
        h[g] = cc * s[0] + kap[g] * s[2];
        const bool wall = g == 0 || g == nk - 1;
        rr[g] = a.qs[I];
        rw[g] = wall ? a.qs[3 * nu + I] : a.qs[3 * nu + I] - dt * (a.gz * s[0] / rbar);
        rt[g] = a.qs[4 * nu + I];
#pragma unroll
        for (int v = 1; v < 3; ++v) {
            const double vs = a.qs[v * nu + I], vc = a.qcur[v * nu + I], vp = a.qprev[v * nu + I];
            a.qprev[v * nu + I] = vc + a.ra * (vp - 2.0 * vc + vs);
            a.qcur[v * nu + I] = vs;
        }
    }
    for (int t = lane; t < nk * GW; t += 64) {
        const int g = t / GW, m = g + t % GW - N;
        Gb[t] = (m >= 0 && m < nk) ? g_entry<N>(a, g, m, izz) : 0.0;
    }
    __syncthreads();
    // r_rho = q*_rho + dt G(rho_bar s_w); r_w += dt G(p_L(s)) / rho_bar (interior)
    for (int g = lane; g < nk; g += 64) {
        double gf = 0.0, gh = 0.0;
#pragma unroll
        for (int d = 0; d < GW; ++d) {
            const int m = g + d - N;
            if (m < 0 || m >= nk) continue;
            gf += Gb[g * GW + d] * f[m];
            gh += Gb[g * GW + d] * h[m];
        }
        rr[g] += dt * gf;
        if (g != 0 && g != nk - 1) rw[g] += dt * gh / rb[g];
    }
    __syncthreads();
    for (int g = lane; g < nk; g += 64) h[g] = c2[g] * rr[g] + kap[g] * rt[g];
    __syncthreads();
    // right-hand side of the w system, and its band matrix
    for (int g = lane; g < nk; g += 64) {
        if (g == 0 || g == nk - 1) {
            x[g] = rw[g];
            continue;
        }
        double gh = 0.0;
#pragma unroll
        for (int d = 0; d < GW; ++d) {
            const int m = g + d - N;
            if (m >= 0 && m < nk) gh += Gb[g * GW + d] * h[m];
        }
        x[g] = rw[g] - dt * gh / rb[g] + dt * a.gz * rr[g] / rb[g];
    }
    const double dt2 = dt * dt;
    for (int t = lane; t < nk * W; t += 64) {
        const int g = t / W, m = g + t % W - B;
        double v = 0.0;
        if (m >= 0 && m < nk) {
            if (g == 0 || g == nk - 1) {
                v = m == g ? 1.0 : 0.0;
            } else {
                double acc = 0.0;  // (G c2 G)_{g m}
                for (int p = g - N; p <= g + N; ++p) {
                    if (p < 0 || p >= nk || m - p < -N || m - p > N) continue;
                    acc += Gb[g * GW + p - g + N] * c2[p] * Gb[p * GW + m - p + N];
                }
                const double gm = (m - g >= -N && m - g <= N) ? Gb[g * GW + m - g + N] : 0.0;
                v = (m == g ? 1.0 : 0.0) - dt2 / rb[g] * acc * rb[m] + dt2 * a.gz / rb[g] * gm * rb[m];
            }
        }
        Ab[t] = v;
    }
    __syncthreads();
    // band LU without pivoting: multipliers stored below the diagonal
    for (int k = 0; k < nk - 1; ++k) {
        const int rmax = k + B < nk - 1 ? k + B : nk - 1;
        if (lane < B && k + 1 + lane <= rmax) {
            const int r = k + 1 + lane;
            Ab[r * W + k - r + B] /= Ab[k * W + B];
        }
        __syncthreads();
        for (int t = lane; t < B * B; t += 64) {
            const int r = k + 1 + t / B, c = k + 1 + t % B;
            if (r <= rmax && c <= rmax)
                Ab[r * W + c - r + B] -= Ab[r * W + k - r + B] * Ab[k * W + c - k + B];
        }
        __syncthreads();
    }
    // forward and back substitution (one lane)
    if (lane == 0) {
        for (int r = 1; r < nk; ++r) {
            double s = x[r];
            for (int c = r - B > 0 ? r - B : 0; c < r; ++c) s -= Ab[r * W + c - r + B] * x[c];
            x[r] = s;
        }
        for (int r = nk - 1; r >= 0; --r) {
            double s = x[r];
            const int cmax = r + B < nk - 1 ? r + B : nk - 1;
            for (int c = r + 1; c <= cmax; ++c) s -= Ab[r * W + c - r + B] * x[c];
            x[r] = s / Ab[r * W + B];
        }
    }
    __syncthreads();
    for (int g = lane; g < nk; g += 64) f[g] = rb[g] * x[g];
    __syncthreads();
    // rho' = r_rho - dt G(rho_bar w), theta' = r_theta; Robert-Asselin filter
    for (int g = lane; g < nk; g += 64) {
        double gf = 0.0;
#pragma unroll
        for (int d = 0; d < GW; ++d) {
            const int m = g + d - N;
            if (m >= 0 && m < nk) gf += Gb[g * GW + d] * f[m];
        }
        const double nv[3] = {rr[g] - dt * gf, x[g], rt[g]};
        const int cv[3] = {0, 3, 4};
        const int64_t I = L + nh * g;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double vc = qc[c * nk + g], vp = qp[c * nk + g];
            a.qprev[cv[c] * nu + I] = vc + a.ra * (vp - 2.0 * vc + nv[c]);
            a.qcur[cv[c] * nu + I] = nv[c];
        }
    }
}

template <int N>
int32_t launch_imex_n(const ImexArgs &a, int64_t lines, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL((k_imex_line<N>), dim3((unsigned)lines), dim3(64), lds, s, a);
    NUMA_HIP(hipGetLastError());
    return NUMA_OK;
}

}  // namespace

uint64_t imex_lds_bytes(const Mesh &m)
{
    const uint64_t nk = (uint64_t)m.d.ne[2] * m.N + 1;
    return 8ull * nk * ((4 * m.N + 1) + (2 * m.N + 1) + 15);
}

int32_t launch_imex_correction(Mesh &m, double dt, double ra, double *qprev, double *qcur, hipStream_t s)
{
    ImexArgs a{};
    a.qs = m.dv.qs;
    a.qcur = qcur;
    a.qprev = qprev;
    a.ref = m.dv.ref;
    a.hcol = m.dv.hcol;
    a.nu = m.nu;
    a.ni = (int)m.ni;
    a.nj = (int)m.nj;
    a.nk = (int)m.nk;
    a.nx = m.d.ne[0];
    a.dt = dt;
    a.ra = ra;
    a.gamma = m.gamma;
    a.gz = -m.ph.g0;
    a.theta0 = m.ph.T0;
    for (int k = 0; k < m.P * m.P; ++k) a.D[k] = m.D[k];
    for (int k = 0; k < m.P; ++k) a.w[k] = m.w[k];
    const size_t lds = (size_t)imex_lds_bytes(m);
    const int64_t lines = m.ni * m.nj;
    switch (m.N) {
    case 1: return launch_imex_n<1>(a, lines, lds, s);
    case 2: return launch_imex_n<2>(a, lines, lds, s);
    case 3: return launch_imex_n<3>(a, lines, lds, s);
    case 4: return launch_imex_n<4>(a, lines, lds, s);
    case 5: return launch_imex_n<5>(a, lines, lds, s);
    case 6: return launch_imex_n<6>(a, lines, lds, s);
    case 7: return launch_imex_n<7>(a, lines, lds, s);
    default: return launch_imex_n<8>(a, lines, lds, s);
    }
}

}  // namespace numa
