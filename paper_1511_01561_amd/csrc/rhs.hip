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
//
// The kernel writes the element-local contributions J w R (the E-vector),
// element-major so that every element writes whole cache lines: in FP64 for
// numa_rhs, and in the contraction precision for the element half of a fused
// stage (the finish kernel sums them).
#include <cmath>

#include "numa_internal.h"

namespace numa {
namespace {

template <typename T>
struct RhsArgs {
    const int32_t *G;  // gather map (shell); the box computes unique ids from its lattice
    const double *q, *ref, *grav;
    const T *met;
    const T *D;
    int64_t nl, nu;
    double gamma, g0;
    int nx, ny;          // box: elements along x and y
    int64_t ni, nj, nk;  // box: lattice extents (x, y periodic)
};

// unique id of local node (i, j, k) of box element e: the element's lattice
// corner plus the local offset, wrapped in the periodic directions
template <int N, typename T>
__device__ __forceinline__ int64_t box_unique(const RhsArgs<T> &a, int64_t e, int i, int j, int k)
{
    const int64_t ex = e % a.nx, ey = (e / a.nx) % a.ny, ez = e / ((int64_t)a.nx * a.ny);
    int64_t gi = ex * N + i, gj = ey * N + j, gk = ez * N + k;
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
    T R[5];     // R_rho', R_u, R_v, R_w, R_theta'
    T Jw;
    int64_t I;  // unique id of the node
    double q[5];
};

// Gathers the element tile, differentiates it and evaluates R at node l of
// element e.  Must be called by all lanes of the block (it synchronises);
// returns false for the padding lanes (l >= (N+1)^3).
template <int N, typename T, bool SHELL>
__device__ __forceinline__ bool element_rhs(const RhsArgs<T> &a, int64_t e, int l, T (*s)[(N + 1) * (N + 1) * (N + 1)],
                                            NodeOut<T> &o)
{
    constexpr int P = N + 1, NP = P * P * P, NF = SHELL ? 9 : 8;
    const bool act = l < NP;
    double rp = 0.0, rho = 1.0, u = 0.0, v = 0.0, w = 0.0, tp = 0.0;
    int64_t I = 0;
    // metric terms do not depend on the tile: load them before the barrier so
    // their latency overlaps the state gather and the equation of state
    T mx[10];
    if (act) {
        const T *mp = a.met + e * 10 * NP + l;
#pragma unroll
        for (int c = 0; c < 10; ++c) mx[c] = mp[c * NP];
    }
    if (act) {
        if constexpr (SHELL) {
            I = a.G[e * NP + l];
        } else {
            constexpr int P_ = N + 1;
            I = box_unique<N, T>(a, e, l % P_, (l / P_) % P_, l / (P_ * P_));
        }
        rp = a.q[I];
        u = a.q[a.nu + I];
        v = a.q[2 * a.nu + I];
        w = a.q[3 * a.nu + I];
        tp = a.q[4 * a.nu + I];
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
    if (!act) return false;
    const int i = l % P, j = (l / P) % P, k = l / (P * P);
    T Di[P], Dj[P], Dk[P];
#pragma unroll
    for (int m = 0; m < P; ++m) {
        Di[m] = a.D[i * P + m];
        Dj[m] = a.D[j * P + m];
        Dk[m] = a.D[k * P + m];
    }
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
        gx = (T)a.grav[I];
        gy = (T)a.grav[a.nu + I];
        gz = (T)a.grav[2 * a.nu + I];
    }
    const T uu = (T)u, vv = (T)v, ww = (T)w;
    o.R[0] = -(dx[0] + dy[1] + dz[2]);
    o.R[1] = -(uu * dx[3] + vv * dy[3] + ww * dz[3]) - dx[7] * irho + buoy * gx;
    o.R[2] = -(uu * dx[4] + vv * dy[4] + ww * dz[4]) - dy[7] * irho + buoy * gy;
    o.R[3] = -(uu * dx[5] + vv * dy[5] + ww * dz[5]) - dz[7] * irho + buoy * gz;
    o.R[4] = -(uu * dx[6] + vv * dy[6] + ww * dz[6]);
    if constexpr (SHELL) o.R[4] -= uu * dx[8] + vv * dy[8] + ww * dz[8];
    o.Jw = mx[9];
    o.I = I;
    o.q[0] = rp;
    o.q[1] = u;
    o.q[2] = v;
    o.q[3] = w;
    o.q[4] = tp;
    return true;
}

template <int N, typename T, typename TO, bool SHELL>
__global__ __launch_bounds__(block_threads<N>()) void k_rhs(RhsArgs<T> a, TO *out)
{
    constexpr int NP = (N + 1) * (N + 1) * (N + 1), NF = SHELL ? 9 : 8;
    __shared__ T s[NF][NP];
    const int64_t e = xcd_remap(blockIdx.x, gridDim.x);
    const int l = threadIdx.x;
    NodeOut<T> o;
    if (!element_rhs<N, T, SHELL>(a, e, l, s, o)) return;
    TO *p = out + e * NP + l;
#pragma unroll
    for (int v = 0; v < 5; ++v) p[v * a.nl] = (TO)(o.Jw * o.R[v]);
}

template <int N, typename T, typename TO>
void launch_n(Mesh &m, const RhsArgs<T> &a, TO *out, hipStream_t s)
{
    dim3 grid((unsigned)m.ne), block(block_threads<N>());
    if (m.d.kind == NUMA_MESH_SHELL) hipLaunchKernelGGL((k_rhs<N, T, TO, true>), grid, block, 0, s, a, out);
    else hipLaunchKernelGGL((k_rhs<N, T, TO, false>), grid, block, 0, s, a, out);
}

template <typename T, typename TO>
void launch_t(Mesh &m, const T *met, const T *D, const double *q, TO *out, hipStream_t s)
{
    RhsArgs<T> a;
    a.G = m.dv.G;
    a.q = q;
    a.ref = m.dv.ref;
    a.grav = m.dv.grav;
    a.met = met;
    a.D = D;
    a.nl = m.nl;
    a.nu = m.nu;
    a.gamma = m.gamma;
    a.g0 = m.ph.g0;
    a.nx = m.d.ne[0];
    a.ny = m.d.ne[1];
    a.ni = m.ni;
    a.nj = m.nj;
    a.nk = m.d.periodic[2] ? m.nk : -1;  // only a periodic z wraps
    switch (m.N) {
    case 1: launch_n<1, T, TO>(m, a, out, s); break;
    case 2: launch_n<2, T, TO>(m, a, out, s); break;
    case 3: launch_n<3, T, TO>(m, a, out, s); break;
    case 4: launch_n<4, T, TO>(m, a, out, s); break;
    case 5: launch_n<5, T, TO>(m, a, out, s); break;
    case 6: launch_n<6, T, TO>(m, a, out, s); break;
    case 7: launch_n<7, T, TO>(m, a, out, s); break;
    default: launch_n<8, T, TO>(m, a, out, s); break;
    }
}

}  // namespace

int32_t launch_rhs(Mesh &m, int32_t prec, const double *q, double *evec, hipStream_t s)
{
    if (prec == NUMA_PREC_MIXED)
        launch_t<float, double>(m, m.dv.met32, m.dv.D32, q, evec, s);
    else
        launch_t<double, double>(m, m.dv.met, m.dv.D64, q, evec, s);
    NUMA_HIP(hipGetLastError());
    return NUMA_OK;
}

// element half of a fused stage: contributions into the workspace E-vector
// (FP32 on the mixed path)
int32_t launch_stage_elements(Mesh &m, int32_t prec, int32_t, double, const double *, const double *qs, double *,
                              hipStream_t s)
{
    if (prec == NUMA_PREC_MIXED)
        launch_t<float, float>(m, m.dv.met32, m.dv.D32, qs, m.dv.ev32, s);
    else
        launch_t<double, double>(m, m.dv.met, m.dv.D64, qs, m.dv.ev64, s);
    NUMA_HIP(hipGetLastError());
    return NUMA_OK;
}

}  // namespace numa
