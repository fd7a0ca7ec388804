// Boyd-Vandeven filter (Sec. "Filter"; Code example 1: after the stages,
// "compute filter", communicate, then DSS with the inverse mass matrix).
//
// Every element's nodal values of the five state variables are transformed to
// Legendre modes, mode k is scaled by sigma_k and the result is transformed
// back: per direction one (N+1) x (N+1) nodal matrix F = V diag(sigma) V^-1,
// applied to the element by sum factorisation (three passes through LDS
// instead of the (N+1)^3 x (N+1)^3 Kronecker product).  The filtered values
// are weighted by J w and summed at the unique nodes (mass-weighted, with the
// wall projection) by the kernels that finish a stage, without the stage
// update.
//
// Modal factors (erfc-log form of the Boyd-Vandeven filter; the paper gives
// neither order p nor cutoff s): sigma_k = 1 for k <= s, else with
// t = (k - s) / (N - s) and d = t - 1/2,
//   sigma_k = erfc(2 sqrt(p) d sqrt(-log(1 - 4 d^2) / (4 d^2))) / 2,
// which is 1/2 at d = 0 and 0 for the top mode.
//
// V^-1 comes from the discrete orthogonality of the Legendre polynomials
// under the GLL rule: sum_i w_i P_j(xi_i) P_k(xi_i) = gamma_k delta_jk with
// gamma_k = 2 / (2k + 1) for k < N and gamma_N = 2 / N (the rule is not exact
// for P_N^2), so V^-1 = diag(1 / gamma) V^T diag(w).
#include <cmath>

#include "kernels.h"

namespace numa {
namespace {

using namespace dev;

struct FilterArgs {
    const int32_t *G;     // [n_elem][np] gather map
    const double *met;    // [n_elem][10][np], J w in component 9
    const double *hcol;   // box: [nx*ny][4][(N+1)^2] column factors, J w_i w_j in factor 0
    const double *q;      // [5][n_unique]
    double *c;            // J w (F q) at every element-local node
    int64_t ne, nl, nu;
    int ni, nj, nk;       // box lattice extents (nk = -1 unless z is periodic)
    FastDiv fx, fy;       // division by the box element counts along x and y
    double w[kMaxP];      // GLL weights
    double F[kMaxP * kMaxP];   // F[i * P + m]
};

// where an element's unique ids and J w come from
enum FilterGeo {
    kGeoStored = 0,   // gather map and stored J w (shell)
    kGeoBox = 1,      // box lattice ids, stored J w
    kGeoBoxCol = 2,   // box lattice ids, J w from the column factors (recomputed metric)
};

template <int N>
constexpr int filter_eb()   // elements per block: about 512 lanes (longer x runs of the gathered rows)
{
    return (N + 1) * (N + 1) * (N + 1) >= 512 ? 1 : 512 / ((N + 1) * (N + 1) * (N + 1));
}

template <int N>
constexpr int filter_threads()
{
    return (filter_eb<N>() * (N + 1) * (N + 1) * (N + 1) + 63) / 64 * 64;
}

// One lane per element-local node; the three directional passes alternate
// between two LDS buffers of the block's elements.  NM: the contributions are
// written node-major ([n_local][5], a copy's five values together, for the box
// and shell finish kernels), staged in LDS so that the block's consecutive
// elements go out as one run of 16-byte stores; else element-major
// ([5][n_local], for the generic DSS).
template <int N, bool NM, int GEO>
__global__ void __launch_bounds__(filter_threads<N>()) k_filter(FilterArgs a)
{
    constexpr int P = N + 1, PP = P * P, NP = PP * P, EB = filter_eb<N>(), NE = EB * NP;
    constexpr int NT = filter_threads<N>();
    __shared__ double Fs[PP];
    __shared__ __align__(16) double s0[5][NE], s1[5][NE];
    const int t = threadIdx.x;
    const int64_t e0 = xcd_remap(blockIdx.x, gridDim.x) * EB;
    if (t < PP) Fs[t] = a.F[t];
    const int le = t / NP, l = t - le * NP;
    const int64_t e = e0 + le;
    const bool on = t < NE && e < a.ne;
    const int i = l % P, j = (l / P) % P, k = l / PP;
    double Jw = 0.0;
    if (on) {
        int64_t g;
        if constexpr (GEO == kGeoStored) {
            g = a.G[e * NP + l];
        } else {   // lattice corner of the element plus the local offset, wrapped where periodic
            const uint32_t ty = fdiv((uint32_t)e, a.fx), ez = fdiv(ty, a.fy);
            const int ex = (int)((uint32_t)e - ty * a.fx.d), ey = (int)(ty - ez * a.fy.d);
            int gi = ex * N + i, gj = ey * N + j, gk = (int)ez * N + k;
            if (gi == a.ni) gi = 0;
            if (gj == a.nj) gj = 0;
            if (gk == a.nk) gk = 0;
            g = gi + (int64_t)a.ni * (gj + (int64_t)a.nj * gk);
            if constexpr (GEO == kGeoBoxCol)
                Jw = a.hcol[(int64_t)(ex + (int)a.fx.d * ey) * (4 * PP) + i + P * j] * a.w[k];
        }
        if constexpr (GEO != kGeoBoxCol) Jw = a.met[(e * 10 + 9) * NP + l];
#pragma unroll
        for (int v = 0; v < 5; ++v) s0[v][t] = a.q[v * a.nu + g];
    } else if (t < NE) {
#pragma unroll
        for (int v = 0; v < 5; ++v) s0[v][t] = 0.0;
    }
    __syncthreads();
    if (t < NE) {   // xi: s1 = F s0 along i
        const int b = t - i;
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            double r = 0.0;
#pragma unroll
            for (int m = 0; m < P; ++m) r = fma(Fs[i * P + m], s0[v][b + m], r);
            s1[v][t] = r;
        }
    }
    __syncthreads();
    if (t < NE) {   // eta: s0 = F s1 along j
        const int b = t - j * P;
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            double r = 0.0;
#pragma unroll
            for (int m = 0; m < P; ++m) r = fma(Fs[j * P + m], s1[v][b + m * P], r);
            s0[v][t] = r;
        }
    }
    __syncthreads();
    double r[5] = {0, 0, 0, 0, 0};
    if (t < NE) {   // zeta along k, times J w
        const int b = t - k * PP;
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            double x = 0.0;
#pragma unroll
            for (int m = 0; m < P; ++m) x = fma(Fs[k * P + m], s0[v][b + m * PP], x);
            r[v] = Jw * x;
        }
    }
    if constexpr (!NM) {
        if (on)
#pragma unroll
            for (int v = 0; v < 5; ++v) a.c[v * a.nl + e * NP + l] = r[v];
    } else {
        // s1 was last read before the previous barrier: reuse it as staging
        double *st = &s1[0][0];
        if (t < NE)
#pragma unroll
            for (int v = 0; v < 5; ++v) st[t * 5 + v] = r[v];
        __syncthreads();
        const int nel = a.ne - e0 < EB ? (int)(a.ne - e0) : EB;
        store_run<double>(a.c + e0 * (NP * 5), st, nel * NP * 5, t, NT);
    }
}

template <int N, int GEO>
void launch_filter_g(const FilterArgs &a, bool node_major, hipStream_t s)
{
    constexpr int EB = filter_eb<N>();
    const unsigned blocks = (unsigned)((a.ne + EB - 1) / EB);
    if (node_major)
        hipLaunchKernelGGL((k_filter<N, true, GEO>), dim3(blocks), dim3(filter_threads<N>()), 0, s, a);
    else
        hipLaunchKernelGGL((k_filter<N, false, GEO>), dim3(blocks), dim3(filter_threads<N>()), 0, s, a);
}

template <int N>
void launch_filter_n(const FilterArgs &a, int geo, bool node_major, hipStream_t s)
{
    if (geo == kGeoStored) launch_filter_g<N, kGeoStored>(a, node_major, s);
    else if (geo == kGeoBox) launch_filter_g<N, kGeoBox>(a, node_major, s);
    else launch_filter_g<N, kGeoBoxCol>(a, node_major, s);
}

// Legendre P_0..P_N at x by the three-term recurrence.
void legendre_row(int N, double x, double *p)
{
    p[0] = 1.0;
    if (N >= 1) p[1] = x;
    for (int k = 1; k < N; ++k) p[k + 1] = ((2 * k + 1) * x * p[k] - k * p[k - 1]) / (k + 1);
}

}  // namespace

void filter_sigma(int N, double order, int32_t cutoff, double *sigma)
{
    for (int k = 0; k <= N; ++k) {
        if (k <= cutoff) {
            sigma[k] = 1.0;
            continue;
        }
        if (k == N) {
            sigma[k] = 0.0;
            continue;
        }
        const double d = (double)(k - cutoff) / (double)(N - cutoff) - 0.5;
        const double chi = d == 0.0 ? 1.0 : std::sqrt(-std::log1p(-4.0 * d * d) / (4.0 * d * d));
        sigma[k] = 0.5 * std::erfc(2.0 * std::sqrt(order) * d * chi);
    }
}

void filter_matrix(int N, const double *xi, const double *w, double order, int32_t cutoff, double *F)
{
    const int P = N + 1;
    double sigma[kMaxP], V[kMaxP][kMaxP], gam[kMaxP];
    filter_sigma(N, order, cutoff, sigma);
    for (int i = 0; i < P; ++i) legendre_row(N, xi[i], V[i]);
    for (int k = 0; k < P; ++k) gam[k] = k < N ? 2.0 / (2 * k + 1) : 2.0 / N;
    for (int i = 0; i < P; ++i)
        for (int c = 0; c < P; ++c) {
            double s = 0.0;
            for (int k = 0; k < P; ++k) s += V[i][k] * sigma[k] / gam[k] * V[c][k];
            F[i * P + c] = s * w[c];
        }
}

int32_t launch_filter(Mesh &m, double order, int32_t cutoff, double *q, hipStream_t s)
{
    FilterArgs a{};
    a.G = m.dv.G;
    a.met = m.dv.met;
    a.hcol = m.dv.hcol;
    a.q = q;
    a.c = m.dv.ev64;
    a.ne = m.ne;
    a.nl = m.nl;
    a.nu = m.nu;
    const bool shell = m.d.kind == NUMA_MESH_SHELL;
    if (!shell) {
        a.ni = (int)m.ni;
        a.nj = (int)m.nj;
        a.nk = m.d.periodic[2] ? (int)m.nk : -1;
        a.fx = fast_div((uint32_t)m.d.ne[0]);
        a.fy = fast_div((uint32_t)m.d.ne[1]);
    }
    for (int k = 0; k < m.P; ++k) a.w[k] = m.w[k];
    filter_matrix(m.N, m.xi, m.w, order, cutoff, a.F);
    if (!shell && filter_split_ok(m)) return launch_filter_split(m, a.F, q, s);
    const int geo = shell ? kGeoStored : (m.metric_mode == NUMA_METRIC_RECOMPUTE ? kGeoBoxCol : kGeoBox);
    // the box (x extent a multiple of the finish segment) and the shell sum
    // node-major contributions with their stage finish kernels; other boxes
    // take the generic DSS
    const bool nm = shell || box_batchable(m);
    switch (m.N) {
    case 1: launch_filter_n<1>(a, geo, nm, s); break;
    case 2: launch_filter_n<2>(a, geo, nm, s); break;
    case 3: launch_filter_n<3>(a, geo, nm, s); break;
    case 4: launch_filter_n<4>(a, geo, nm, s); break;
    case 5: launch_filter_n<5>(a, geo, nm, s); break;
    case 6: launch_filter_n<6>(a, geo, nm, s); break;
    case 7: launch_filter_n<7>(a, geo, nm, s); break;
    default: launch_filter_n<8>(a, geo, nm, s); break;
    }
    NUMA_HIP(hipGetLastError());
    if (shell) return launch_shell_plain_finish(m, m.dv.ev64, q, s);
    if (nm) return launch_box_plain_finish(m, m.dv.ev64, q, s);
    return launch_dss(m, 5, m.dv.ev64, q, NUMA_DSS_MASS | NUMA_DSS_NOFLUX, s, stage_minv(m));
}

}  // namespace numa
