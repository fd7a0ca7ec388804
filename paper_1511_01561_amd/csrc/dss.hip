// Direct stiffness summation, mass-matrix inverse, no-flux projection and the
// SSP-RK3 stage update (the pointwise part of each stage in Code example 1:
// "DSS and multiply with inverse mass matrix", "update q").
//
// The summation is a gather over the inverse of the element -> unique map:
// each unique node sums its element-local copies in ascending order.  No
// atomics, no colouring and no barriers are needed, and the result does not
// depend on scheduling (the paper avoids atomics by re-ordering elements and
// adding barriers; a gather removes the race altogether).
#include "kernels.h"

namespace numa {
namespace {

using namespace dev;

__global__ void k_dss(PointArgs p, int nvar, const double *cin, double *out, int flags)
{
    int64_t I = xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (I >= p.nu) return;
    const int32_t b = p.off[I], en = p.off[I + 1];
    double r[5] = {0, 0, 0, 0, 0};
    const bool mass = flags & NUMA_DSS_MASS;
    const double mi = mass ? p.Minv[I] : 1.0;
    for (int v0 = 0; v0 < nvar; v0 += 5) {
        int nv = nvar - v0 < 5 ? nvar - v0 : 5;
        for (int v = 0; v < nv; ++v) r[v] = 0.0;
        for (int32_t c = b; c < en; ++c) {
            int64_t cc = p.idx[c];
            for (int v = 0; v < nv; ++v) r[v] += cin[(v0 + v) * p.nl + cc];
        }
        if (mass)
            for (int v = 0; v < nv; ++v) r[v] *= mi;
        if ((flags & NUMA_DSS_NOFLUX) && nvar == 5) noflux(p, I, r[1], r[2], r[3]);
        for (int v = 0; v < nv; ++v) out[(v0 + v) * p.nu + I] = r[v];
    }
}

__global__ void k_rk_stage(int64_t n, StageCoef c, const double *qn, const double *qs, const double *r,
                           double *qout)
{
    int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    qout[a] = rk_update(c, c.a == 0.0 ? 0.0 : qn[a], qs[a], r[a]);
}

// Second half of a fused stage: DSS (mass-weighted), no-flux projection and
// the stage update of every unique node.  Lanes walk the nodes in
// first-occurrence order of the element scan (own[]), so a block gathers the
// contributions of a few adjacent elements that its XCD has just read, and
// its state reads and writes merge into whole cache lines across consecutive
// blocks.  Copies are summed in ascending element-local order.  qout may alias
// qs or qn (one lane per node).
template <typename T>
__global__ void k_stage_finish(PointArgs p, const int32_t *own, const int32_t *toff, const int32_t *tidx,
                               const T *ev, StageCoef c, const double *qn, const double *qs, double *qout)
{
    int64_t t = xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (t >= p.nu) return;
    const int64_t I = own[t];
    const int32_t b = toff[t], en = toff[t + 1];
    double r[5] = {0, 0, 0, 0, 0};
    for (int32_t c = b; c < en; ++c) {
        const int64_t cc = tidx[c];
#pragma unroll
        for (int v = 0; v < 5; ++v) r[v] += (double)ev[v * p.nl + cc];
    }
    const double mi = p.Minv[I];
#pragma unroll
    for (int v = 0; v < 5; ++v) r[v] *= mi;
    noflux(p, I, r[1], r[2], r[3]);
#pragma unroll
    for (int v = 0; v < 5; ++v)
        qout[v * p.nu + I] = rk_update(c, c.a == 0.0 ? 0.0 : qn[v * p.nu + I], qs[v * p.nu + I], r[v]);
}

// Finish of a fused stage on the shell: one lane per unique node in unique
// order I = h + n_h gk, so state reads and writes run along the horizontal
// numbering.  The copies of a node factor: its horizontal copies in the
// bottom layer (hoff/hidx, 1 to 4, ascending) times its radial copies (local
// k = 0 of layer gk/N and k = N of the layer below on a layer boundary, else
// one).  The contributions are node-major [n_local][5]; the up to four
// horizontal copies of one radial copy are loaded together (absent ones are
// not loaded).  PLAIN: the
// output is the summed, mass-weighted, projected value (the filter's DSS).
struct ShellFin {
    const int32_t *hoff, *hidx;
    FastDiv fnh;      // division by n_horiz
    int nz;           // element layers
    int64_t layer;    // elements of one layer times (N+1)^3
};

// fold: the contributions away from the bottom and top layers are
// J w (q_s + cdt R) (k_rhs), so M^-1 times their sum is y = q_s + cdt R and
// q_s is not read there (as in box_finish_node)
template <int N, typename T, bool PLAIN = false>
__global__ void k_shell_finish(PointArgs p, ShellFin sf, const T *ev, StageCoef c, int fold, const double *qn,
                               const double *qs, double *qout)
{
    constexpr int P = N + 1, PP = P * P;
    const int64_t t = xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (t >= p.nu) return;
    const int32_t I = (int32_t)t;
    const uint32_t gk = fdiv((uint32_t)I, sf.fnh);
    const int32_t h = I - (int32_t)(gk * sf.fnh.d);
    const double *qsi = qs + I, *qni = qn + I;
    const double mi = p.Minv[I];
    const int top = sf.nz * N;
    const bool folded = !PLAIN && fold && gk != 0 && gk != (uint32_t)top;
    double qsv[5] = {0, 0, 0, 0, 0}, qnv[5] = {0, 0, 0, 0, 0};
    if (!PLAIN)
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            qsv[v] = folded ? 0.0 : qsi[v * p.nu];
            qnv[v] = c.a == 0.0 ? 0.0 : qni[v * p.nu];
        }
    // radial copies: (layer, local k)
    int ez[2], kz[2], nzc = 1;
    if (gk == (uint32_t)top) {
        ez[0] = sf.nz - 1;
        kz[0] = N;
    } else {
        ez[0] = (int)(gk / N);
        kz[0] = (int)(gk - (uint32_t)ez[0] * N);
        if (kz[0] == 0 && ez[0] > 0) {
            ez[1] = ez[0] - 1;
            kz[1] = N;
            nzc = 2;
        }
    }
    const int32_t hb = sf.hoff[h], hn = sf.hoff[h + 1] - hb;
    int32_t hc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) hc[q] = sf.hidx[hb + (q < hn ? q : hn - 1)];
    double r[5] = {0, 0, 0, 0, 0};
    for (int z = 0; z < nzc; ++z) {
        const int64_t base = ez[z] * sf.layer + PP * kz[z];
        T c[4][5];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const T *src = ev + (base + hc[q]) * 5;
            if (q < hn) {  // absent copies are not loaded
#pragma unroll
                for (int v = 0; v < 5; ++v) c[q][v] = src[v];
            } else {
#pragma unroll
                for (int v = 0; v < 5; ++v) c[q][v] = (T)0;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int v = 0; v < 5; ++v) r[v] += q < hn ? (double)c[q][v] : 0.0;
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) r[v] *= mi;
    double *qoi = qout + I;
    if (folded) {
#pragma unroll
        for (int v = 0; v < 5; ++v) qoi[v * p.nu] = rk_update_folded(c, qnv[v], r[v]);
        return;
    }
    noflux(p, I, r[1], r[2], r[3]);
#pragma unroll
    for (int v = 0; v < 5; ++v) qoi[v * p.nu] = PLAIN ? r[v] : rk_update(c, qnv[v], qsv[v], r[v]);
}

inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <typename T, bool PLAIN = false>
void launch_shell_finish_t(Mesh &m, const T *ev, const StageCoef &c, const double *qn, const double *qs,
                           double *qout, hipStream_t s, int fold = 0)
{
    PointArgs p = point_args(m);
    if (!PLAIN) p.Minv = stage_minv(m);  // the shell filter takes the stored J w
    ShellFin sf;
    sf.hoff = m.dv.hoff;
    sf.hidx = m.dv.hidx;
    sf.fnh = fast_div((uint32_t)m.nh);
    sf.nz = m.d.ne[2];
    sf.layer = 6 * (int64_t)m.d.ne[0] * m.d.ne[0] * m.np;
    const dim3 grid(nblocks(m.nu, 256)), block(256);
    switch (m.N) {
    case 1: hipLaunchKernelGGL((k_shell_finish<1, T, PLAIN>), grid, block, 0, s, p, sf, ev, c, fold, qn, qs, qout); break;
    case 2: hipLaunchKernelGGL((k_shell_finish<2, T, PLAIN>), grid, block, 0, s, p, sf, ev, c, fold, qn, qs, qout); break;
    case 3: hipLaunchKernelGGL((k_shell_finish<3, T, PLAIN>), grid, block, 0, s, p, sf, ev, c, fold, qn, qs, qout); break;
    case 4: hipLaunchKernelGGL((k_shell_finish<4, T, PLAIN>), grid, block, 0, s, p, sf, ev, c, fold, qn, qs, qout); break;
    case 5: hipLaunchKernelGGL((k_shell_finish<5, T, PLAIN>), grid, block, 0, s, p, sf, ev, c, fold, qn, qs, qout); break;
    case 6: hipLaunchKernelGGL((k_shell_finish<6, T, PLAIN>), grid, block, 0, s, p, sf, ev, c, fold, qn, qs, qout); break;
    case 7: hipLaunchKernelGGL((k_shell_finish<7, T, PLAIN>), grid, block, 0, s, p, sf, ev, c, fold, qn, qs, qout); break;
    default: hipLaunchKernelGGL((k_shell_finish<8, T, PLAIN>), grid, block, 0, s, p, sf, ev, c, fold, qn, qs, qout); break;
    }
}

}  // namespace

int32_t launch_dss(Mesh &m, int32_t nvar, const double *cin, double *out, int32_t flags, hipStream_t s,
                   const double *minv)
{
    PointArgs p = point_args(m);
    if (minv) p.Minv = minv;
    hipLaunchKernelGGL(k_dss, dim3(nblocks(m.nu, 256)), dim3(256), 0, s, p, nvar, cin, out, flags);
    NUMA_HIP(hipGetLastError());
    return NUMA_OK;
}

StageCoef ssp33_stage(int stage, double dt)
{
    if (stage == 0) return StageCoef{0.0, 1.0, dt};
    if (stage == 1) return StageCoef{0.75, 0.25, dt};
    return StageCoef{1.0 / 3.0, 2.0 / 3.0, dt};
}

int32_t launch_rk_stage(Mesh &m, int32_t stage, double dt, const double *qn, const double *qs, const double *r,
                        double *qout, hipStream_t s)
{
    int64_t n = 5 * m.nu;
    hipLaunchKernelGGL(k_rk_stage, dim3(nblocks(n, 256)), dim3(256), 0, s, n, ssp33_stage(stage, dt), qn, qs, r,
                       qout);
    NUMA_HIP(hipGetLastError());
    return NUMA_OK;
}

int32_t launch_shell_plain_finish(Mesh &m, const double *ev, double *q, hipStream_t s)
{
    launch_shell_finish_t<double, true>(m, ev, StageCoef{0.0, 1.0, 0.0}, nullptr, nullptr, q, s);
    NUMA_HIP(hipGetLastError());
    return NUMA_OK;
}

int32_t launch_stage_finish(Mesh &m, int32_t prec, const StageCoef &c, const double *qn, const double *qs,
                            double *qout, hipStream_t s)
{
    if (m.d.kind == NUMA_MESH_SHELL) {  // node-major contributions (launch_stage_elements)
        if (prec == NUMA_PREC_MIXED)
            launch_shell_finish_t<float>(m, m.dv.ev32, c, qn, qs, qout, s);
        else
            launch_shell_finish_t<double>(m, m.dv.ev64, c, qn, qs, qout, s, shell_folds(m, prec, c) ? 1 : 0);
        NUMA_HIP(hipGetLastError());
        return NUMA_OK;
    }
    PointArgs p = point_args(m);
    p.Minv = stage_minv(m);
    if (prec == NUMA_PREC_MIXED)
        hipLaunchKernelGGL(k_stage_finish<float>, dim3(nblocks(m.nu, 256)), dim3(256), 0, s, p, m.dv.own, m.dv.toff,
                           m.dv.tidx, m.dv.ev32, c, qn, qs, qout);
    else
        hipLaunchKernelGGL(k_stage_finish<double>, dim3(nblocks(m.nu, 256)), dim3(256), 0, s, p, m.dv.own, m.dv.toff,
                           m.dv.tidx, m.dv.ev64, c, qn, qs, qout);
    NUMA_HIP(hipGetLastError());
    return NUMA_OK;
}

}  // namespace numa
