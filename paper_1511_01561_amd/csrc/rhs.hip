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

#include "kernels.h"

namespace numa {
namespace {

using namespace dev;

// NM: node-major output [n_local][5] (the element's 5 (N+1)^3 values staged
// through the tile and written as one contiguous run), for the shell's fused
// stage; otherwise element-major [5][n_local].
template <int N, typename T, typename TO, bool SHELL, int GEO, bool NM = false>
__global__ __launch_bounds__(block_threads<N>()) void k_rhs(RhsArgs<T> a, TO *out)
{
    constexpr int NP = (N + 1) * (N + 1) * (N + 1), NF = SHELL ? 9 : 8, BT = block_threads<N>();
    __shared__ T s[NF][NP];
    const int64_t e = xcd_remap(blockIdx.x, gridDim.x);
    const int l = threadIdx.x;
    NodeOut<T> o;
    if constexpr (NM) {
        static_assert(sizeof(TO) == sizeof(T), "node-major output is staged in the tile");
        // element_rhs, with the node's state kept for the fold
        NodeIn<T> in;
        node_gather<N, T, SHELL, GEO>(a, e, l, in);
        node_stage<N, T, SHELL, GEO>(a, e, l, in, s);
        __syncthreads();
        const bool act = l < NP;
        if (act) {
            T Di[N + 1], Dj[N + 1], Dk[N + 1];
            d_rows<N, T>(a.D, l, Di, Dj, Dk);
            node_derive<N, T, SHELL, GEO>(a, l, in, Di, Dj, Dk, s, o);
        }
        __syncthreads();  // every lane has finished reading the tile
        TO *st = (TO *)&s[0][0];
        if (act) {
            // J w R, or J w (q_s + cdt R) away from the bottom and top layers
            const int ez = (int)fdiv((uint32_t)e, a.feh), k = l / ((N + 1) * (N + 1));
            const bool wall = (ez == 0 && k == 0) || (ez == a.nz - 1 && k == N);
            if (sizeof(T) == 8 && a.fold && !wall) {
                const double qv[5] = {in.rp, in.u, in.v, in.w, in.tp};
#pragma unroll
                for (int v = 0; v < 5; ++v) st[l * 5 + v] = (TO)(o.Jw * fma((T)a.cdt, o.R[v], (T)qv[v]));
            } else {
#pragma unroll
                for (int v = 0; v < 5; ++v) st[l * 5 + v] = (TO)(o.Jw * o.R[v]);
            }
        }
        __syncthreads();
        TO *dst = out + e * (NP * 5);
#pragma unroll
        for (int r = 0; r < (NP * 5 + BT - 1) / BT; ++r) {
            const int t = l + r * BT;
            if (t < NP * 5) dst[t] = st[t];
        }
    } else {
        const bool act = element_rhs<N, T, SHELL, GEO>(a, e, l, s, o);
        if (!act) return;
        TO *p = out + e * NP + l;
#pragma unroll
        for (int v = 0; v < 5; ++v) p[v * a.nl] = (TO)(o.Jw * o.R[v]);
    }
}

template <int N, typename T, typename TO>
void launch_n(Mesh &m, const RhsArgs<T> &a, TO *out, bool node_major, hipStream_t s)
{
    dim3 grid((unsigned)m.ne), block(block_threads<N>());
    if constexpr (sizeof(TO) == sizeof(T)) {
        if (node_major && m.d.kind == NUMA_MESH_SHELL) {
            if (m.metric_mode == NUMA_METRIC_RECOMPUTE)
                hipLaunchKernelGGL((k_rhs<N, T, TO, true, kMetricShell, true>), grid, block, 0, s, a, out);
            else
                hipLaunchKernelGGL((k_rhs<N, T, TO, true, kMetricStored, true>), grid, block, 0, s, a, out);
            return;
        }
    }
    if (m.d.kind == NUMA_MESH_SHELL && m.metric_mode == NUMA_METRIC_RECOMPUTE)
        hipLaunchKernelGGL((k_rhs<N, T, TO, true, kMetricShell>), grid, block, 0, s, a, out);
    else if (m.d.kind == NUMA_MESH_SHELL)
        hipLaunchKernelGGL((k_rhs<N, T, TO, true, kMetricStored>), grid, block, 0, s, a, out);
    else if (m.metric_mode == NUMA_METRIC_RECOMPUTE)
        hipLaunchKernelGGL((k_rhs<N, T, TO, false, kMetricBox>), grid, block, 0, s, a, out);
    else
        hipLaunchKernelGGL((k_rhs<N, T, TO, false, kMetricStored>), grid, block, 0, s, a, out);
}

template <typename T, typename TO>
void launch_t(Mesh &m, const T *met, const T *D, const double *q, TO *out, bool node_major, hipStream_t s,
              double cdt = 0.0, int fold = 0)
{
    RhsArgs<T> a;
    a.cdt = cdt;
    a.fold = fold;
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
    a.hcol = m.dv.hcol;
    a.nx = m.d.ne[0];
    a.ny = m.d.ne[1];
    a.nz = m.d.ne[2];
    a.fx = fast_div((uint32_t)m.d.ne[0]);
    a.fy = fast_div((uint32_t)m.d.ne[1]);
    a.scol = m.dv.scol;
    a.slay = m.dv.slay;
    a.shid = m.dv.shid;
    a.nh = m.nh;
    a.feh = fast_div((uint32_t)(m.d.kind == NUMA_MESH_SHELL ? 6 * m.d.ne[0] * m.d.ne[0] : 1));
    if (m.d.kind == NUMA_MESH_BOX) a.bm = box_metric(m);
    eos_coeffs(m.gamma, a.eos);
    a.xi = m.dv.xi64;
    a.w = m.dv.w64;
    a.Dd = m.dv.D64;
    a.ni = (int)m.ni;
    a.nj = (int)m.nj;
    a.nk = m.d.periodic[2] ? (int)m.nk : -1;  // only a periodic z wraps
    switch (m.N) {
    case 1: launch_n<1, T, TO>(m, a, out, node_major, s); break;
    case 2: launch_n<2, T, TO>(m, a, out, node_major, s); break;
    case 3: launch_n<3, T, TO>(m, a, out, node_major, s); break;
    case 4: launch_n<4, T, TO>(m, a, out, node_major, s); break;
    case 5: launch_n<5, T, TO>(m, a, out, node_major, s); break;
    case 6: launch_n<6, T, TO>(m, a, out, node_major, s); break;
    case 7: launch_n<7, T, TO>(m, a, out, node_major, s); break;
    default: launch_n<8, T, TO>(m, a, out, node_major, s); break;
    }
}

}  // namespace

int32_t launch_rhs(Mesh &m, int32_t prec, const double *q, double *evec, hipStream_t s)
{
    if (prec == NUMA_PREC_MIXED)
        launch_t<float, double>(m, m.dv.met32, m.dv.D32, q, evec, false, s);
    else
        launch_t<double, double>(m, m.dv.met, m.dv.D64, q, evec, false, s);
    NUMA_HIP(hipGetLastError());
    return NUMA_OK;
}

// element half of a fused stage: contributions into the workspace E-vector
// (FP32 on the mixed path)
int32_t launch_stage_elements(Mesh &m, int32_t prec, const StageCoef &c, const double *qs, hipStream_t s)
{
    // the shell's finish reads node-major contributions, the generic one element-major
    const bool nm = m.d.kind == NUMA_MESH_SHELL;
    if (prec == NUMA_PREC_MIXED)
        launch_t<float, float>(m, m.dv.met32, m.dv.D32, qs, m.dv.ev32, nm, s);
    else
        launch_t<double, double>(m, m.dv.met, m.dv.D64, qs, m.dv.ev64, nm, s, c.cdt, shell_folds(m, prec, c) ? 1 : 0);
    NUMA_HIP(hipGetLastError());
    return NUMA_OK;
}

}  // namespace numa
