// Element-wise right-hand side (the paper's create_rhs): Eq. (discstrongform)
// with the derivatives of Eq. (derivatives) (chain rule through the metric).
//
// One workgroup per element, one lane per element-local node.  The unique
// state is gathered through the element -> unique map, the equation of state
// is evaluated in FP64, and the eight differentiated fields
//   rho u, rho v, rho w, u, v, w, theta', p'   (+ theta_bar on the shell)
// are staged once in LDS so that all fields are differentiated from one tile
// (the paper's "all derivatives of an element in one matrix per direction").
// Each lane keeps its three rows of the derivative matrix in registers.
#include <cmath>

#include "numa_internal.h"

namespace numa {
namespace {

template <typename T>
struct RhsArgs {
    const int32_t *G;
    const double *q, *ref, *grav;
    const T *met;
    const T *D;
    double *out;
    int64_t nl, nu;
    double gamma, g0;
};

template <int N>
constexpr int block_threads() { return (((N + 1) * (N + 1) * (N + 1) + 63) / 64) * 64; }

template <int N, typename T, bool SHELL>
__global__ __launch_bounds__(block_threads<N>()) void k_rhs(RhsArgs<T> a)
{
    constexpr int P = N + 1, NP = P * P * P, NF = SHELL ? 9 : 8;
    __shared__ T s[NF][NP];
    const int64_t e = blockIdx.x;
    const int l = threadIdx.x;
    const bool act = l < NP;
    double rp = 0.0, rho = 1.0, u = 0.0, v = 0.0, w = 0.0;
    if (act) {
        const int64_t I = a.G[e * NP + l];
        rp = a.q[I];
        u = a.q[a.nu + I];
        v = a.q[2 * a.nu + I];
        w = a.q[3 * a.nu + I];
        const double tp = a.q[4 * a.nu + I];
        const double rb = a.ref[I], tb = a.ref[a.nu + I], pb = a.ref[2 * a.nu + I];
        rho = rb + rp;
        // p' = p_bar ((rho theta / rho_bar theta_bar)^gamma - 1) without cancellation
        const double dl = rp * tb + rb * tp + rp * tp;
        const double pp = pb * expm1(a.gamma * log1p(dl / (rb * tb)));
        s[0][l] = (T)(rho * u);
        s[1][l] = (T)(rho * v);
        s[2][l] = (T)(rho * w);
        s[3][l] = (T)u;
        s[4][l] = (T)v;
        s[5][l] = (T)w;
        s[6][l] = (T)tp;
        s[7][l] = (T)pp;
        if constexpr (SHELL) {
            // the background theta is differentiated relative to the element's first node
            const double t0 = a.ref[a.nu + a.G[e * NP]];
            s[8][l] = (T)(tb - t0);
        }
    }
    __syncthreads();
    if (!act) return;
    const int i = l % P, j = (l / P) % P, k = l / (P * P);
    T Di[P], Dj[P], Dk[P];
#pragma unroll
    for (int m = 0; m < P; ++m) {
        Di[m] = a.D[i * P + m];
        Dj[m] = a.D[j * P + m];
        Dk[m] = a.D[k * P + m];
    }
    const T *mp = a.met + e * 10 * NP + l;
    T mx[10];
#pragma unroll
    for (int c = 0; c < 10; ++c) mx[c] = mp[c * NP];
    T dx[NF], dy[NF], dz[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        T da = 0, db = 0, dc = 0;
#pragma unroll
        for (int m = 0; m < P; ++m) {
            da += Di[m] * s[f][m + P * (j + P * k)];
            db += Dj[m] * s[f][i + P * (m + P * k)];
            dc += Dk[m] * s[f][i + P * (j + P * m)];
        }
        dx[f] = da * mx[0] + db * mx[3] + dc * mx[6];
        dy[f] = da * mx[1] + db * mx[4] + dc * mx[7];
        dz[f] = da * mx[2] + db * mx[5] + dc * mx[8];
    }
    const T irho = (T)(1.0 / rho);
    const T buoy = (T)(rp / rho);
    T gx = 0, gy = 0, gz = (T)(-a.g0);
    if constexpr (SHELL) {
        const int64_t I = a.G[e * NP + l];
        gx = (T)a.grav[I];
        gy = (T)a.grav[a.nu + I];
        gz = (T)a.grav[2 * a.nu + I];
    }
    const T uu = (T)u, vv = (T)v, ww = (T)w;
    T R0 = -(dx[0] + dy[1] + dz[2]);
    T R1 = -(uu * dx[3] + vv * dy[3] + ww * dz[3]) - dx[7] * irho + buoy * gx;
    T R2 = -(uu * dx[4] + vv * dy[4] + ww * dz[4]) - dy[7] * irho + buoy * gy;
    T R3 = -(uu * dx[5] + vv * dy[5] + ww * dz[5]) - dz[7] * irho + buoy * gz;
    T R4 = -(uu * dx[6] + vv * dy[6] + ww * dz[6]);
    if constexpr (SHELL) R4 -= uu * dx[8] + vv * dy[8] + ww * dz[8];
    const T Jw = mx[9];
    double *o = a.out + e * NP + l;
    o[0] = (double)(Jw * R0);
    o[a.nl] = (double)(Jw * R1);
    o[2 * a.nl] = (double)(Jw * R2);
    o[3 * a.nl] = (double)(Jw * R3);
    o[4 * a.nl] = (double)(Jw * R4);
}

template <int N, typename T>
void launch_rhs_n(Mesh &m, const T *met, const T *D, const double *q, double *evec, hipStream_t s)
{
    RhsArgs<T> a;
    a.G = m.dv.G;
    a.q = q;
    a.ref = m.dv.ref;
    a.grav = m.dv.grav;
    a.met = met;
    a.D = D;
    a.out = evec;
    a.nl = m.nl;
    a.nu = m.nu;
    a.gamma = m.gamma;
    a.g0 = m.ph.g0;
    if (m.d.kind == NUMA_MESH_SHELL)
        hipLaunchKernelGGL((k_rhs<N, T, true>), dim3((unsigned)m.ne), dim3(block_threads<N>()), 0, s, a);
    else
        hipLaunchKernelGGL((k_rhs<N, T, false>), dim3((unsigned)m.ne), dim3(block_threads<N>()), 0, s, a);
}

template <typename T>
void launch_rhs_t(Mesh &m, const T *met, const T *D, const double *q, double *evec, hipStream_t s)
{
    switch (m.N) {
    case 1: launch_rhs_n<1, T>(m, met, D, q, evec, s); break;
    case 2: launch_rhs_n<2, T>(m, met, D, q, evec, s); break;
    case 3: launch_rhs_n<3, T>(m, met, D, q, evec, s); break;
    case 4: launch_rhs_n<4, T>(m, met, D, q, evec, s); break;
    case 5: launch_rhs_n<5, T>(m, met, D, q, evec, s); break;
    case 6: launch_rhs_n<6, T>(m, met, D, q, evec, s); break;
    case 7: launch_rhs_n<7, T>(m, met, D, q, evec, s); break;
    default: launch_rhs_n<8, T>(m, met, D, q, evec, s); break;
    }
}

}  // namespace

int32_t launch_rhs(Mesh &m, int32_t prec, const double *q, double *evec, hipStream_t s)
{
    if (prec == NUMA_PREC_MIXED)
        launch_rhs_t<float>(m, m.dv.met32, m.dv.D32, q, evec, s);
    else
        launch_rhs_t<double>(m, m.dv.met, m.dv.D64, q, evec, s);
    NUMA_HIP(hipGetLastError());
    return NUMA_OK;
}

}  // namespace numa
