// Direct stiffness summation, mass-matrix inverse, no-flux projection and the
// SSP-RK3 stage update (the pointwise part of each stage in Code example 1:
// "DSS and multiply with inverse mass matrix", "update q").
//
// The summation is a gather over the inverse of the element -> unique map:
// each unique node sums its element-local copies in ascending order.  No
// atomics, no colouring and no barriers are needed, and the result does not
// depend on scheduling (the paper avoids atomics by re-ordering elements and
// adding barriers; a gather removes the race altogether).
#include <type_traits>

#include "numa_internal.h"

namespace numa {
namespace {

struct PointArgs {
    const int32_t *off, *idx;
    const double *Minv, *nrm;
    int64_t nl, nu, nh;
    int walls;
};

PointArgs point_args(const Mesh &m)
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

__device__ inline double rk_combine(int stage, double qn, double y)
{
    if (stage == 0) return y;
    if (stage == 1) return 0.75 * qn + 0.25 * y;
    return (1.0 / 3.0) * qn + (2.0 / 3.0) * y;
}

__global__ void k_rk_stage(int64_t n, int stage, double dt, const double *qn, const double *qs,
                           const double *r, double *qout)
{
    int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    double y = qs[a] + dt * r[a];
    qout[a] = rk_combine(stage, stage == 0 ? 0.0 : qn[a], y);
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
                               const T *ev, int stage, double dt, const double *qn, const double *qs, double *qout)
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
    for (int v = 0; v < 5; ++v) {
        double y = qs[v * p.nu + I] + dt * r[v];
        qout[v * p.nu + I] = rk_combine(stage, stage == 0 ? 0.0 : qn[v * p.nu + I], y);
    }
}

// Finish of a fused stage on the box.  A block takes SEG consecutive elements
// along x of one (ey, ez) and, per element, the lattice nodes whose lower
// corner it is (local 0 <= i, j, k < N); lanes run along x fastest, so every
// state read and write covers SEG*N consecutive unique ids.  The copies of a
// node follow from its lattice position: on an element face along a
// direction it has two copies (local index 0 of the element above and N of
// the one below, wrapped when periodic), else one.  A second launch with
// kbase = N, klayers = 1 covers the top wall layer.
struct BoxFin {
    int nx, ny, nz, walls;
    int64_t ni, nj, nk;
};

template <int N, int SEG, typename T>
__global__ void k_box_finish(PointArgs p, BoxFin b, const T *ev, int kbase, int klayers, int stage, double dt,
                             const double *qn, const double *qs, double *qout)
{
    constexpr int P = N + 1, NP = P * P * P, W = SEG * N;
    const int lane = threadIdx.x;
    if (lane >= W * N * klayers) return;
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t nseg = b.nx / SEG;
    const int64_t sx = blk % nseg, ey = (blk / nseg) % b.ny, ez = kbase == 0 ? blk / (nseg * b.ny) : b.nz - 1;
    const int a = lane % W, jj = (lane / W) % N, kk = lane / (W * N);
    const int64_t gi = sx * W + a, gj = ey * N + jj, gk = ez * N + kbase + kk;
    const int64_t I = gi + b.ni * (gj + b.nj * gk);
    // copies along each direction: (element index along the direction, local index)
    int64_t cx[2], cy[2], cz[2];
    int lx[2], ly[2], lz[2], nxc, nyc, nzc;
    const int64_t exa = gi / N;
    if (a % N == 0) {  // gi is a multiple of N: element face in x
        cx[0] = exa; lx[0] = 0;
        cx[1] = exa == 0 ? b.nx - 1 : exa - 1; lx[1] = N;
        nxc = 2;
    } else {
        cx[0] = exa; lx[0] = (int)(gi - exa * N);
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
    double r[5] = {0, 0, 0, 0, 0};
    for (int z = 0; z < nzc; ++z)
        for (int y = 0; y < nyc; ++y)
            for (int x = 0; x < nxc; ++x) {
                const int64_t e = cx[x] + b.nx * (cy[y] + b.ny * cz[z]);
                const int64_t c = e * NP + lx[x] + P * (ly[y] + P * lz[z]);
#pragma unroll
                for (int v = 0; v < 5; ++v) r[v] += (double)ev[v * p.nl + c];
            }
    const double mi = p.Minv[I];
#pragma unroll
    for (int v = 0; v < 5; ++v) r[v] *= mi;
    noflux(p, I, r[1], r[2], r[3]);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        double y = qs[v * p.nu + I] + dt * r[v];
        qout[v * p.nu + I] = rk_combine(stage, stage == 0 ? 0.0 : qn[v * p.nu + I], y);
    }
}

inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <int N, int SEG, typename T>
void launch_box_finish_t(Mesh &m, const T *ev, int stage, double dt, const double *qn, const double *qs, double *qout,
                         hipStream_t s)
{
    BoxFin b;
    b.nx = m.d.ne[0];
    b.ny = m.d.ne[1];
    b.nz = m.d.ne[2];
    b.walls = m.walls ? 1 : 0;
    b.ni = m.ni;
    b.nj = m.nj;
    b.nk = m.nk;
    const int threads = ((SEG * N * N * N + 63) / 64) * 64;
    const int64_t nb = (int64_t)(b.nx / SEG) * b.ny * b.nz;
    hipLaunchKernelGGL((k_box_finish<N, SEG, T>), dim3((unsigned)nb), dim3(threads), 0, s, point_args(m), b, ev, 0, N,
                       stage, dt, qn, qs, qout);
    if (m.walls) {
        const int tthreads = ((SEG * N * N + 63) / 64) * 64;
        hipLaunchKernelGGL((k_box_finish<N, SEG, T>), dim3((unsigned)((b.nx / SEG) * b.ny)), dim3(tthreads), 0, s,
                           point_args(m), b, ev, N, 1, stage, dt, qn, qs, qout);
    }
}

// x-segment length: whole 128-byte lines of FP64 state where the block fits
template <int N>
constexpr int seg_for() { return 4 * N * N * N <= 1024 ? 4 : (2 * N * N * N <= 1024 ? 2 : 1); }

template <typename T>
bool launch_box_finish(Mesh &m, const T *ev, int stage, double dt, const double *qn, const double *qs, double *qout,
                       hipStream_t s)
{
    auto go = [&](auto nt) {
        constexpr int N = decltype(nt)::value;
        constexpr int SEG = seg_for<N>();
        if (m.d.ne[0] % SEG) return false;
        launch_box_finish_t<N, SEG, T>(m, ev, stage, dt, qn, qs, qout, s);
        return true;
    };
    switch (m.N) {
    case 1: return go(std::integral_constant<int, 1>());
    case 2: return go(std::integral_constant<int, 2>());
    case 3: return go(std::integral_constant<int, 3>());
    case 4: return go(std::integral_constant<int, 4>());
    case 5: return go(std::integral_constant<int, 5>());
    case 6: return go(std::integral_constant<int, 6>());
    case 7: return go(std::integral_constant<int, 7>());
    default: return go(std::integral_constant<int, 8>());
    }
}

}  // namespace

int32_t launch_dss(Mesh &m, int32_t nvar, const double *cin, double *out, int32_t flags, hipStream_t s)
{
    hipLaunchKernelGGL(k_dss, dim3(nblocks(m.nu, 256)), dim3(256), 0, s, point_args(m), nvar, cin, out, flags);
    NUMA_HIP(hipGetLastError());
    return NUMA_OK;
}

int32_t launch_rk_stage(Mesh &m, int32_t stage, double dt, const double *qn, const double *qs, const double *r,
                        double *qout, hipStream_t s)
{
    int64_t n = 5 * m.nu;
    hipLaunchKernelGGL(k_rk_stage, dim3(nblocks(n, 256)), dim3(256), 0, s, n, stage, dt, qn, qs, r, qout);
    NUMA_HIP(hipGetLastError());
    return NUMA_OK;
}

int32_t launch_stage_finish(Mesh &m, int32_t prec, int32_t stage, double dt, const double *qn, const double *qs,
                            double *qout, hipStream_t s)
{
    if (m.d.kind == NUMA_MESH_BOX) {
        bool done = prec == NUMA_PREC_MIXED ? launch_box_finish<float>(m, m.dv.ev32, stage, dt, qn, qs, qout, s)
                                            : launch_box_finish<double>(m, m.dv.ev64, stage, dt, qn, qs, qout, s);
        if (done) {
            NUMA_HIP(hipGetLastError());
            return NUMA_OK;
        }
    }
    if (prec == NUMA_PREC_MIXED)
        hipLaunchKernelGGL(k_stage_finish<float>, dim3(nblocks(m.nu, 256)), dim3(256), 0, s, point_args(m), m.dv.own,
                           m.dv.toff, m.dv.tidx, m.dv.ev32, stage, dt, qn, qs, qout);
    else
        hipLaunchKernelGGL(k_stage_finish<double>, dim3(nblocks(m.nu, 256)), dim3(256), 0, s, point_args(m), m.dv.own,
                           m.dv.toff, m.dv.tidx, m.dv.ev64, stage, dt, qn, qs, qout);
    NUMA_HIP(hipGetLastError());
    return NUMA_OK;
}

}  // namespace numa
