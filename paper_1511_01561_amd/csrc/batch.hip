// Batched fused stages on box meshes: the elements and nodes of several
// independent solves of the same order advance together, one element launch
// and one finish launch per stage for the whole batch (continuous batching of
// ensemble members and regional solves).  Each item brings its own state and
// private scratch; geometry may be shared between items.  The per-element
// and per-node arithmetic is the single-mesh code (kernels.h), so an item's
// result does not depend on what it is batched with.  A single box mesh
// (numa_step) runs through the same kernels with one item.
#include "kernels.h"

#include <vector>

namespace numa {
namespace {

using namespace dev;

constexpr int kMaxBatch = 16;  // items per launch (kernel-argument table)

struct BatchItem {
    const double *qs;  // stage input state [5][nu]
    double *qout;      // stage output state
    const double *qn;  // reference state of the stage update (q^n or an earlier stage)
    const double *ref, *Minv, *nrm;
    const void *met;      // [ne][10][np] of T
    void *ev;             // [nl][5] of T: contributions of this stage, node-major
    const double *hcol;   // column factors of the recomputed metric
    int32_t *flag;        // non-finite flag of the item's state, or null
    int nu, nh;           // unique nodes, per level (meshes are limited to 32-bit indices)
    int ni, nj, nkw;      // lattice extents; nkw: extent in z when periodic, else -1
    int nz, walls;
    int ne;               // elements
    int mblk;             // finish blocks of the main layers: (nx/SEG) ny nz
    FastDiv fx, fy, fseg;  // division by nx, ny and nx/SEG (colour passes: fseg by nx/2, fy by ny/2)
    double cdt;            // (beta / b) dt of the stage update
    double theta0;         // the box reference is isentropic: theta_bar = theta0 everywhere
    BoxMetric bm;          // constants of the recomputed metric
    int eoff, boff;        // first element / finish block of this item in the launch (eoff: a
                           // multiple of the elements per element workgroup)
};

struct Batch {
    int n;
    int fold;       // the column kernel folds q_s into the contributions (box_finish_node)
    double ca, cb;  // weights of the reference state and of the stage in the update (same for all items)
    double gamma, g0;
    const void *D;
    const double *xi, *w, *Dd;  // FP64 GLL nodes, weights, derivative matrix
    double eos[kEosTerms];
    BatchItem it[kMaxBatch];
};
static_assert(sizeof(Batch) <= 4096, "the batch table must fit the kernel arguments");

// item of launch-wide block g (items are in ascending eoff / boff order)
__device__ __forceinline__ int batch_item(const Batch &B, int g, bool fin)
{
    int k = 0;
    while (k + 1 < B.n && g >= (fin ? B.it[k + 1].boff : B.it[k + 1].eoff)) ++k;
    return k;
}

// element-kernel arguments of one batch item
template <typename T>
__device__ __forceinline__ RhsArgs<T> elem_args(const Batch &B, const BatchItem &it)
{
    RhsArgs<T> a;
    a.G = nullptr;
    a.q = it.qs;
    a.ref = it.ref;
    a.grav = nullptr;
    a.met = (const T *)it.met;
    a.D = (const T *)B.D;
    a.hcol = it.hcol;
    a.nl = 0;
    a.nu = it.nu;
    a.gamma = B.gamma;
    a.g0 = B.g0;
    a.nx = (int)it.fx.d;
    a.ny = (int)it.fy.d;
    a.nz = it.nz;
    a.ni = it.ni;
    a.nj = it.nj;
    a.nk = it.nkw;
    a.fx = it.fx;
    a.fy = it.fy;
    a.scol = nullptr;
    a.slay = nullptr;
    a.shid = nullptr;
    a.nh = it.nh;
    a.feh = FastDiv{1, 1, 0, 0};
    a.bm = it.bm;
#pragma unroll
    for (int c = 0; c < kEosTerms; ++c) a.eos[c] = B.eos[c];
    a.xi = B.xi;
    a.w = B.w;
    a.Dd = B.Dd;
    return a;
}

// node-major [n_local][5] output of element e (a copy's five values in one
// run for the finish), staged through LDS (st, 5 (N+1)^3 values) so that the
// block writes them as one contiguous, coalesced run; the caller has
// synchronised after writing st
template <int N, typename T>
__device__ __forceinline__ void store_contributions(const BatchItem &it, int e, int l, const T *st)
{
    constexpr int NP = (N + 1) * (N + 1) * (N + 1), BT = block_threads<N>();
    T *out = (T *)it.ev + (int64_t)e * (NP * 5);
#pragma unroll
    for (int r = 0; r < (NP * 5 + BT - 1) / BT; ++r) {
        const int t = l + r * BT;
        if (t < NP * 5) out[t] = st[t];
    }
}

// One workgroup per element (the launch-wide element index, XCD-remapped).
template <int N, typename T, int GEO>
__global__ __launch_bounds__(block_threads<N>()) void k_elem_batch(Batch B)
{
    constexpr int NP = (N + 1) * (N + 1) * (N + 1);
    __shared__ T s[8][NP];
    const int g = (int)xcd_remap(blockIdx.x, gridDim.x);
    const BatchItem &it = B.it[batch_item(B, g, false)];
    const int e = g - it.eoff;
    const RhsArgs<T> a = elem_args<T>(B, it);
    NodeOut<T> o;
    const int l = threadIdx.x;
    // element_rhs, with the node's state kept for the fold
    NodeIn<T> in;
    node_gather<N, T, false, GEO>(a, e, l, in);
    node_stage<N, T, false, GEO>(a, e, l, in, s);
    __syncthreads();
    const bool act = l < NP;
    if (act) {
        if constexpr (GEO == kMetricBox) {  // FP64 at N = 7, 8: R direction by direction
            node_derive_box_dirs<N, T>(a, l, in, s, o);
        } else {
            T Di[N + 1], Dj[N + 1], Dk[N + 1];
            d_rows<N, T>(a.D, l, Di, Dj, Dk);
            node_derive<N, T, false, GEO>(a, l, in, Di, Dj, Dk, s, o);
        }
    }
    __syncthreads();  // every lane has finished reading the tile
    T *st = &s[0][0];
    if (act) {
        const int k = l / ((N + 1) * (N + 1));
        const bool wall = it.walls && ((in.ez == 0 && k == 0) || (in.ez == it.nz - 1 && k == N));
        if (sizeof(T) == 8 && B.fold && !wall) {  // J w (q_s + cdt R), as in k_elem_col
            const double qv[5] = {in.rp, in.u, in.v, in.w, in.tp};
#pragma unroll
            for (int v = 0; v < 5; ++v) st[l * 5 + v] = o.Jw * fma((T)it.cdt, o.R[v], (T)qv[v]);
        } else {
#pragma unroll
            for (int v = 0; v < 5; ++v) st[l * 5 + v] = o.Jw * o.R[v];
        }
    }
    __syncthreads();
    store_contributions<N, T>(it, e, l, st);
}

// Column variant for the recomputed box metric: a workgroup takes EB
// consecutive elements and a lane one (i, j) column of one of them, i.e. the
// N+1 nodes (i, j, 0..N).  The lane gathers its column (all loads in flight
// together), evaluates the equation of state and keeps the column's fields in
// registers: the zeta derivatives are contractions with D_km, which is the
// same for every lane, so they need no LDS.  Only the xi and eta derivatives
// read the element tile.  The arithmetic per node is that of element_rhs.
// Elements per workgroup: as many columns as fill four wavefronts up to
// N = 4 (ten x-consecutive elements at N = 4: longer contiguous runs in the
// gather and the store, measured ~1 % faster than two wavefronts), two
// wavefronts for the streaming variant at N = 5, 6 (its larger tile would
// leave one wavefront per SIMD), one element at N = 7 and 8; the tile (8
// fields of (N+1)^3 nodes per element) stays within 80 KB.
template <int N, typename T>
constexpr int col_eb()
{
    constexpr int PP = (N + 1) * (N + 1);
    return N >= 7 ? 1 : (N <= 4 ? 256 / PP : 128 / PP);
}
template <int N, typename T>
constexpr int col_threads() { return ((col_eb<N, T>() * (N + 1) * (N + 1) + 63) / 64) * 64; }
// workgroups per CU the column kernel is compiled for: in FP32 at N = 4 the
// tile (40 KB) lets four share a CU if the registers fit 4 waves per SIMD
template <int N, typename T>
constexpr int col_blocks() { return (sizeof(T) == 4 && N == 4) ? 4 : 1; }

// MODE 0: write J w R node-major for the finish kernel (NUMA_STAGE_GATHER);
// MODE 1: one colour pass of NUMA_STAGE_COLOUR: the workgroup's elements are
// the elements of colour `colour` (parity of ex, ey, ez), EB consecutive ones
// along x, and every lane adds its nodes' J w R to the FP64 accumulator with
// a plain read-modify-write (no other element of the colour has the node).
template <int N, typename T, int MODE = 0>
__global__ __launch_bounds__((col_threads<N, T>()), (col_blocks<N, T>())) void k_elem_col(Batch B, int colour)
{
    constexpr int P = N + 1, PP = P * P, NP = PP * P, EB = col_eb<N, T>(), BT = col_threads<N, T>();
    __shared__ T s[EB][8][NP];
    const int g0 = (int)xcd_remap(blockIdx.x, gridDim.x) * EB;
    const BatchItem &it = B.it[batch_item(B, g0, false)];
    const RhsArgs<T> a = elem_args<T>(B, it);
    const int e0 = g0 - it.eoff;  // first element of the workgroup in the item
    const int t = threadIdx.x, q = t / PP, c = t % PP, i = c % P, j = c / P;
    const bool act = q < EB && e0 + q < it.ne;
    // per node of the column: 1/rho and rho'/rho (formed in FP64; in FP64
    // rho' itself is kept and rho'/rho formed where it is used, the same
    // product), zeta derivatives of the 8 tile fields
    constexpr bool F64 = sizeof(T) == 8;
    T irho[P], buoy[P], dz[8][P];
    double c0 = 0.0, c1 = 0.0, c2 = 0.0, c3 = 0.0;
    int ez = 0, base = 0;
    const int layer = a.ni * a.nj;
    if (act) {
        BoxElem be;
        if constexpr (MODE == 1) {
            const uint32_t ec = (uint32_t)(e0 + q), t1 = fdiv(ec, it.fseg), t2 = fdiv(t1, it.fy);
            be.ex = 2 * (int)(ec - t1 * it.fseg.d) + (colour & 1);
            be.ey = 2 * (int)(t1 - t2 * it.fy.d) + ((colour >> 1) & 1);
            be.ez = 2 * (int)t2 + (colour >> 2);
        } else {
            be = box_elem((uint32_t)(e0 + q), a.fx, a.fy);
        }
        ez = be.ez;
        const double *cp = a.hcol + (int64_t)(be.ex + a.nx * be.ey) * (4 * PP) + c;
        c0 = cp[0];
        c1 = cp[PP];
        c2 = cp[2 * PP];
        c3 = cp[3 * PP];
        int gi = be.ex * N + i, gj = be.ey * N + j;
        if (gi == a.ni) gi = 0;
        if (gj == a.nj) gj = 0;
        base = gi + a.ni * gj;
        T col[8][P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            int gk = be.ez * N + k;
            if (gk == a.nk) gk = 0;
            const int32_t I = base + layer * gk;
            const double *qp = a.q + I, *rf = a.ref + I;
            const double rp = qp[0], u = qp[a.nu], v = qp[2 * a.nu], w = qp[3 * a.nu], tp = qp[4 * a.nu];
            const double rb = rf[0], tb = it.theta0, pb = rf[2 * a.nu];
            const double rho = rb + rp;
            // p' = p_bar ((rho theta / rho_bar theta_bar)^gamma - 1) without cancellation
            const double dl = rp * tb + rb * tp + rp * tp;
            const double pp = pb * eos_rel(dl / (rb * tb), a.gamma, a.eos);
            const double ir = 1.0 / rho;
            irho[k] = (T)ir;
            buoy[k] = F64 ? (T)rp : (T)(rp * ir);
            col[0][k] = (T)(rho * u);
            col[1][k] = (T)(rho * v);
            col[2][k] = (T)(rho * w);
            col[3][k] = (T)u;
            col[4][k] = (T)v;
            col[5][k] = (T)w;
            col[6][k] = (T)tp;
            col[7][k] = (T)pp;
#pragma unroll
            for (int f = 0; f < 8; ++f) s[q][f][c + PP * k] = col[f][k];
        }
        const T *D = a.D;
#pragma unroll
        for (int f = 0; f < 8; ++f)
#pragma unroll
            for (int k = 0; k < P; ++k) {
                T d = 0;
#pragma unroll
                for (int m = 0; m < P; ++m) d += D[k * P + m] * col[f][m];
                dz[f][k] = d;
            }
    }
    __syncthreads();  // tiles complete
    T res[P][5];
    if (act) {
        T Di[P], Dj[P];
#pragma unroll
        for (int m = 0; m < P; ++m) {
            Di[m] = a.D[i * P + m];
            Dj[m] = a.D[j * P + m];
        }
#pragma unroll
        for (int k = 0; k < P; ++k) {
            T mx[10];
            box_node_metric<T>(a.bm, ez, B.xi[k], c0 * B.w[k], c1, c2, c3, mx);
            T dd[8][3];
#pragma unroll
            for (int f = 0; f < 8; ++f) {
                T da = 0, db = 0;
#pragma unroll
                for (int m = 0; m < P; ++m) {
                    da += Di[m] * s[q][f][m + P * (j + P * k)];
                    db += Dj[m] * s[q][f][i + P * (m + P * k)];
                }
                dd[f][0] = da;
                dd[f][1] = db;
                dd[f][2] = dz[f][k];
            }
            const int l = c + PP * k;
            // node_combine with 1/rho and rho'/rho already formed
            const T uu = s[q][3][l], vv = s[q][4][l], ww = s[q][5][l];
            T Uc[3];
            Uc[0] = uu * mx[0];
            Uc[1] = vv * mx[4];
            Uc[2] = uu * mx[6] + vv * mx[7] + ww * mx[8];
            auto cart = [&](int f, int cc) -> T {
                if (cc == 0) return dd[f][0] * mx[0] + dd[f][2] * mx[6];
                if (cc == 1) return dd[f][1] * mx[4] + dd[f][2] * mx[7];
                return dd[f][2] * mx[8];
            };
            auto adv = [&](int f) -> T { return Uc[0] * dd[f][0] + Uc[1] * dd[f][1] + Uc[2] * dd[f][2]; };
            const T gz = (T)(-a.g0);
            const T bk = F64 ? buoy[k] * irho[k] : buoy[k];
            T R[5];
            R[0] = -(cart(0, 0) + cart(1, 1) + cart(2, 2));
            R[1] = -adv(3) - cart(7, 0) * irho[k];
            R[2] = -adv(4) - cart(7, 1) * irho[k];
            R[3] = -adv(5) - cart(7, 2) * irho[k] + bk * gz;
            R[4] = -adv(6);
            // J w R, or J w (q_s + cdt R) away from the walls when folding
            const bool wall = it.walls && ((ez == 0 && k == 0) || (ez == a.nz - 1 && k == N));
            if (F64 && B.fold && !wall) {
                const T qv[5] = {buoy[k], uu, vv, ww, s[q][6][l]};
#pragma unroll
                for (int v = 0; v < 5; ++v) res[k][v] = mx[9] * fma((T)it.cdt, R[v], qv[v]);
            } else {
#pragma unroll
                for (int v = 0; v < 5; ++v) res[k][v] = mx[9] * R[v];
            }
        }
    }
    if constexpr (MODE == 1) {
        if (act) {
            double *acc = (double *)it.ev;
#pragma unroll
            for (int k = 0; k < P; ++k) {
                int gk = ez * N + k;
                if (gk == a.nk) gk = 0;
                const int32_t I = base + layer * gk;
#pragma unroll
                for (int v = 0; v < 5; ++v) acc[I + v * a.nu] += (double)res[k][v];
            }
        }
        return;  // every lane: no barrier follows
    }
    __syncthreads();  // tiles read
    T *st = &s[0][0][0];
    if (act) {
#pragma unroll
        for (int k = 0; k < P; ++k)
#pragma unroll
            for (int v = 0; v < 5; ++v) st[(q * NP + c + PP * k) * 5 + v] = res[k][v];
    }
    __syncthreads();
    // the workgroup's elements are consecutive: one contiguous run
    const int ne = it.ne - e0 < EB ? it.ne - e0 : EB;
    T *out = (T *)it.ev + (int64_t)e0 * (NP * 5);
    store_run<T>(out, st, ne * NP * 5, t, BT);
}

// NUMA_STAGE_COLOUR: zero the accumulator [5][nu] of every item (a kernel,
// not a memset: the stage may be captured in a graph)
__global__ void k_colour_zero(Batch B)
{
    const int g = (int)blockIdx.x;
    const BatchItem &it = B.it[batch_item(B, g, true)];
    const int64_t I = (int64_t)(g - it.boff) * 256 + threadIdx.x;
    if (I >= it.nu) return;
    double *acc = (double *)it.ev;
#pragma unroll
    for (int v = 0; v < 5; ++v) acc[I + v * it.nu] = 0.0;
}

// NUMA_STAGE_COLOUR: M^-1, wall projection and stage update of every unique
// node from the accumulated sum (the tail of box_finish_node)
__global__ void k_colour_finish(Batch B)
{
    const int g = (int)xcd_remap(blockIdx.x, gridDim.x);
    const BatchItem &it = B.it[batch_item(B, g, true)];
    const int64_t I = (int64_t)(g - it.boff) * 256 + threadIdx.x;
    if (I >= it.nu) return;
    const double *acc = (const double *)it.ev;
    const StageCoef sc{B.ca, B.cb, it.cdt};
    const double mi = it.Minv[I];
    const bool wall = it.walls && (I < it.nh || I >= it.nu - it.nh);
    double r[5], qnv[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        r[v] = acc[I + v * it.nu] * mi;
        qnv[v] = sc.a == 0.0 ? 0.0 : it.qn[I + v * it.nu];
    }
    double o[5];
    if (B.fold && !wall) {
#pragma unroll
        for (int v = 0; v < 5; ++v) it.qout[I + v * it.nu] = o[v] = rk_update_folded(sc, qnv[v], r[v]);
        flag_nonfinite(it.flag, o, 5);
        return;
    }
    PointArgs p;
    p.off = nullptr;
    p.idx = nullptr;
    p.Minv = it.Minv;
    p.nrm = it.nrm;
    p.nl = 0;
    p.nu = it.nu;
    p.nh = it.nh;
    p.walls = it.walls;
    noflux(p, I, r[1], r[2], r[3]);
#pragma unroll
    for (int v = 0; v < 5; ++v) it.qout[I + v * it.nu] = o[v] = rk_update(sc, qnv[v], it.qs[I + v * it.nu], r[v]);
    flag_nonfinite(it.flag, o, 5);
}

// Streaming variant of the column kernel: after the tile is built the lane
// walks the 8 fields once, reads its own column of each field (the zeta
// contraction), the xi and eta lines of each of its nodes, and adds the
// field's terms to the R of its N+1 nodes, so that only R, the advecting
// contravariant velocity and 1/rho, rho'/rho of the column stay in registers
// (the terms are added in the order element_rhs sums them).
template <int N, typename T>
__global__ __launch_bounds__((col_threads<N, T>())) void k_elem_stream(Batch B)
{
    constexpr int P = N + 1, PP = P * P, NP = PP * P, EB = col_eb<N, T>(), BT = col_threads<N, T>();
    __shared__ T s[EB][8][NP];
    const int g0 = (int)xcd_remap(blockIdx.x, gridDim.x) * EB;
    const BatchItem &it = B.it[batch_item(B, g0, false)];
    const RhsArgs<T> a = elem_args<T>(B, it);
    const int e0 = g0 - it.eoff;
    const int t = threadIdx.x, q = t / PP, c = t % PP, i = c % P, j = c / P;
    const bool act = q < EB && e0 + q < it.ne;
    T irho[P], buoy[P], Uc[P][3];
    double c0 = 0.0, c1 = 0.0, c2 = 0.0, c3 = 0.0;
    int ez = 0;
    if (act) {
        const BoxElem be = box_elem((uint32_t)(e0 + q), a.fx, a.fy);
        ez = be.ez;
        const double *cp = a.hcol + (int64_t)(be.ex + a.nx * be.ey) * (4 * PP) + c;
        c0 = cp[0];
        c1 = cp[PP];
        c2 = cp[2 * PP];
        c3 = cp[3 * PP];
        int gi = be.ex * N + i, gj = be.ey * N + j;
        if (gi == a.ni) gi = 0;
        if (gj == a.nj) gj = 0;
        const int base = gi + a.ni * gj, layer = a.ni * a.nj;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            int gk = be.ez * N + k;
            if (gk == a.nk) gk = 0;
            const int32_t I = base + layer * gk;
            const double *qp = a.q + I, *rf = a.ref + I;
            const double rp = qp[0], u = qp[a.nu], v = qp[2 * a.nu], w = qp[3 * a.nu], tp = qp[4 * a.nu];
            const double rb = rf[0], tb = it.theta0, pb = rf[2 * a.nu];
            const double rho = rb + rp;
            // p' = p_bar ((rho theta / rho_bar theta_bar)^gamma - 1) without cancellation
            const double dl = rp * tb + rb * tp + rp * tp;
            const double pp = pb * eos_rel(dl / (rb * tb), a.gamma, a.eos);
            const double ir = 1.0 / rho;
            irho[k] = (T)ir;
            buoy[k] = (T)(rp * ir);
            T mx[10];
            box_node_metric<T>(a.bm, ez, B.xi[k], c0, c1, c2, c3, mx);
            const T uu = (T)u, vv = (T)v, ww = (T)w;
            Uc[k][0] = uu * mx[0];
            Uc[k][1] = vv * mx[4];
            Uc[k][2] = uu * mx[6] + vv * mx[7] + ww * mx[8];
            const int l = c + PP * k;
            s[q][0][l] = (T)(rho * u);
            s[q][1][l] = (T)(rho * v);
            s[q][2][l] = (T)(rho * w);
            s[q][3][l] = uu;
            s[q][4][l] = vv;
            s[q][5][l] = ww;
            s[q][6][l] = (T)tp;
            s[q][7][l] = (T)pp;
        }
    }
    __syncthreads();  // tiles complete
    T R[P][5];
    if (act) {
        T Di[P], Dj[P];
#pragma unroll
        for (int m = 0; m < P; ++m) {
            Di[m] = a.D[i * P + m];
            Dj[m] = a.D[j * P + m];
        }
        const T *D = a.D;
        const T mx0 = (T)a.bm.ixa, mx4 = (T)a.bm.iyb, mx8 = (T)c1;
#pragma unroll
        for (int f = 0; f < 8; ++f) {
            T cf[P];
#pragma unroll
            for (int m = 0; m < P; ++m) cf[m] = s[q][f][c + PP * m];
#pragma unroll
            for (int k = 0; k < P; ++k) {
                const double omz = 1.0 - ((double)ez + 0.5 * (1.0 + B.xi[k])) * a.bm.inz;  // 1 - z/H
                const T mx6 = (T)(omz * c2), mx7 = (T)(omz * c3);
                T dc = 0, da = 0, db = 0;
#pragma unroll
                for (int m = 0; m < P; ++m) dc += D[k * P + m] * cf[m];
                if (f != 1 && f != 2) {
#pragma unroll
                    for (int m = 0; m < P; ++m) da += Di[m] * s[q][f][m + P * (j + P * k)];
                }
                if (f != 0 && f != 2) {
#pragma unroll
                    for (int m = 0; m < P; ++m) db += Dj[m] * s[q][f][i + P * (m + P * k)];
                }
                if (f == 0) R[k][0] = da * mx0 + dc * mx6;                // d(rho u)/dx
                if (f == 1) R[k][0] = R[k][0] + (db * mx4 + dc * mx7);    // + d(rho v)/dy
                if (f == 2) R[k][0] = -(R[k][0] + dc * mx8);              // + d(rho w)/dz
                if (f >= 3 && f <= 6) R[k][f - 2] = -(Uc[k][0] * da + Uc[k][1] * db + Uc[k][2] * dc);
                if (f == 7) {
                    R[k][1] = R[k][1] - (da * mx0 + dc * mx6) * irho[k];
                    R[k][2] = R[k][2] - (db * mx4 + dc * mx7) * irho[k];
                    R[k][3] = R[k][3] - (dc * mx8) * irho[k] + buoy[k] * (T)(-a.g0);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const T jw = (T)(c0 * B.w[k]);
#pragma unroll
            for (int v = 0; v < 5; ++v) R[k][v] = jw * R[k][v];
        }
    }
    __syncthreads();  // tiles read
    T *st = &s[0][0][0];
    if (act) {
#pragma unroll
        for (int k = 0; k < P; ++k)
#pragma unroll
            for (int v = 0; v < 5; ++v) st[(q * NP + c + PP * k) * 5 + v] = R[k][v];
    }
    __syncthreads();
    // the workgroup's elements are consecutive: one contiguous run
    const int ne = it.ne - e0 < EB ? it.ne - e0 : EB;
    T *out = (T *)it.ev + (int64_t)e0 * (NP * 5);
    store_run<T>(out, st, ne * NP * 5, t, BT);
}

template <int N, int SEG, typename T, bool PLAIN = false>
__global__ void k_fin_batch(Batch B)
{
    const int g = (int)xcd_remap(blockIdx.x, gridDim.x);
    const BatchItem &it = B.it[batch_item(B, g, true)];
    int lb = g - it.boff;
    int kbase = 0, klayers = N;
    if (lb >= it.mblk) {  // the top wall layer
        kbase = N;
        klayers = 1;
        lb -= it.mblk;
    }
    const uint32_t t = fdiv((uint32_t)lb, it.fseg);
    const int sx = lb - (int)(t * it.fseg.d);
    const uint32_t ez = fdiv(t, it.fy);
    const int ey = (int)(t - ez * it.fy.d);
    PointArgs p;
    p.off = nullptr;
    p.idx = nullptr;
    p.Minv = it.Minv;
    p.nrm = it.nrm;
    p.nl = 0;
    p.nu = it.nu;
    p.nh = it.nh;
    p.walls = it.walls;
    BoxFin b;
    b.nx = (int)it.fx.d;
    b.ny = (int)it.fy.d;
    b.nz = it.nz;
    b.walls = it.walls;
    b.ni = it.ni;
    b.nj = it.nj;
    b.fold = B.fold;
    box_finish_node<N, SEG, T, PLAIN>(p, b, (const T *)it.ev, sx, ey, kbase == 0 ? (int)ez : it.nz - 1, threadIdx.x,
                                      kbase, klayers, StageCoef{B.ca, B.cb, it.cdt}, it.qn, it.qs, it.qout,
                                      PLAIN ? nullptr : it.flag);
}

template <int N, typename T, int SEG>
int32_t run_chunk_seg(const StepItem *items, int n, int phase, hipStream_t s, bool colour)
{
    Batch B;
    B.n = n;
    B.ca = items[0].c.a;
    B.cb = items[0].c.b;
    B.gamma = items[0].mesh->gamma;
    B.g0 = items[0].mesh->ph.g0;
    B.D = std::is_same<T, float>::value ? (const void *)items[0].mesh->dv.D32 : (const void *)items[0].mesh->dv.D64;
    B.xi = items[0].mesh->dv.xi64;
    B.w = items[0].mesh->dv.w64;
    B.Dd = items[0].mesh->dv.D64;
    eos_coeffs(B.gamma, B.eos);
    // the recomputed metric runs a column kernel, EB elements per workgroup:
    // registers for every field's column up to N = 4, the streaming variant
    // above (FP64 at N = 7, 8 outgrows both: one node per lane there)
    constexpr int kind = N <= 4 ? 0 : (sizeof(T) == 4 || N <= 6 ? 1 : 2);
    constexpr bool col_ok = kind != 2;
    const bool recompute = items[0].mesh->metric_mode == NUMA_METRIC_RECOMPUTE;
    const bool col = recompute && col_ok;
    const int eb = col ? col_eb<N, T>() : 1;
    // FP64 update that uses q_s (b != 0): the column and one-node-per-lane
    // element kernels fold q_s into the contributions (the streaming one,
    // which runs at its register limit, does not)
    B.fold = (std::is_same<T, double>::value && B.cb != 0.0 && !(recompute && kind == 1)) ? 1 : 0;
    int64_t eo = 0, bo = 0;
    for (int k = 0; k < n; ++k) {
        const Mesh &m = *items[k].mesh;
        BatchItem &it = B.it[k];
        it.qs = items[k].qs;
        it.qout = items[k].qout;
        it.qn = items[k].qn;
        it.ref = m.dv.ref;
        it.Minv = stage_minv(m);
        it.nrm = m.dv.nrm;
        it.met = std::is_same<T, float>::value ? (const void *)m.dv.met32 : (const void *)m.dv.met;
        it.ev = items[k].ev;
        it.hcol = m.dv.hcol;
        it.flag = items[k].flag;
        it.nu = (int)m.nu;
        it.nh = (int)m.nh;
        it.ni = (int)m.ni;
        it.nj = (int)m.nj;
        it.nkw = m.d.periodic[2] ? (int)m.nk : -1;
        it.nz = m.d.ne[2];
        it.walls = m.walls ? 1 : 0;
        it.fx = fast_div((uint32_t)m.d.ne[0]);
        it.fy = fast_div((uint32_t)m.d.ne[1]);
        it.fseg = fast_div((uint32_t)(m.d.ne[0] / SEG));
        const int64_t mblk = (int64_t)(m.d.ne[0] / SEG) * m.d.ne[1] * m.d.ne[2];
        it.mblk = (int)mblk;
        it.cdt = items[k].c.cdt;
        it.theta0 = m.ph.T0;
        it.bm = box_metric(m);
        it.ne = (int)m.ne;
        it.eoff = (int)eo;
        it.boff = (int)bo;
        if (colour) {  // a colour pass covers ne/8 elements; the pointwise kernels 256 nodes per block
            it.ne = (int)(m.ne / 8);
            it.fseg = fast_div((uint32_t)(m.d.ne[0] / 2));
            it.fy = fast_div((uint32_t)(m.d.ne[1] / 2));
            eo += (it.ne + eb - 1) / eb * eb;
            bo += (m.nu + 255) / 256;
        } else {
            eo += (m.ne + eb - 1) / eb * eb;
            bo += mblk + (m.walls ? (int64_t)(m.d.ne[0] / SEG) * m.d.ne[1] : 0);
        }
    }
    if (eo >= (int64_t(1) << 31) || bo >= (int64_t(1) << 31)) {
        set_error("batch: more than 2^31 - 1 elements in one launch");
        return NUMA_EUNSUPPORTED;
    }
    for (int k = n; k < kMaxBatch; ++k) B.it[k] = BatchItem{};
    if (colour) {
        if constexpr (kind == 0) {
            if (phase == 0) {
                hipLaunchKernelGGL(k_colour_zero, dim3((unsigned)bo), dim3(256), 0, s, B);
                for (int c = 0; c < 8; ++c)
                    hipLaunchKernelGGL((k_elem_col<N, T, 1>), dim3((unsigned)(eo / eb)), dim3(col_threads<N, T>()), 0, s,
                                       B, c);
            } else {
                hipLaunchKernelGGL(k_colour_finish, dim3((unsigned)bo), dim3(256), 0, s, B);
            }
            NUMA_HIP(hipGetLastError());
            return NUMA_OK;
        }
    }
    if (phase == 0) {
        if (!recompute) {
            hipLaunchKernelGGL((k_elem_batch<N, T, kMetricStored>), dim3((unsigned)eo), dim3(block_threads<N>()), 0, s,
                               B);
        } else if constexpr (kind == 0) {
            hipLaunchKernelGGL((k_elem_col<N, T>), dim3((unsigned)(eo / eb)), dim3(col_threads<N, T>()), 0, s, B, 0);
        } else if constexpr (kind == 1) {
            hipLaunchKernelGGL((k_elem_stream<N, T>), dim3((unsigned)(eo / eb)), dim3(col_threads<N, T>()), 0, s, B);
        } else {
            hipLaunchKernelGGL((k_elem_batch<N, T, kMetricBox>), dim3((unsigned)eo), dim3(block_threads<N>()), 0, s, B);
        }
    } else {
        const int threads = ((SEG * N * N * N + 63) / 64) * 64;
        hipLaunchKernelGGL((k_fin_batch<N, SEG, T>), dim3((unsigned)bo), dim3(threads), 0, s, B);
    }
    NUMA_HIP(hipGetLastError());
    return NUMA_OK;
}

// The finish segment of a launch: the widest (seg_wide) that divides the x
// element count of every item, halving down to seg_for, which divides every
// batchable mesh's.  At N = 3 a 4-element segment is 12 lattice points, 96 of
// every 128 bytes of a state line; 16 elements are 48 points, three whole
// lines (measured at 64x64x16: finish 82 -> 61 us).  The per-node code and
// its order of the copies do not depend on the segment: results are the
// same bit for bit whichever segment a launch takes.
template <int N> constexpr int seg_wide() { return N == 3 ? 16 : seg_for<N>(); }

template <int N>
int pick_seg(const StepItem *items, int n)
{
    int seg = seg_wide<N>();
    for (int k = 0; k < n; ++k)
        while (seg > seg_for<N>() && items[k].mesh->d.ne[0] % seg) seg /= 2;
    return seg;
}

template <int N, typename T>
int32_t run_chunk(const StepItem *items, int n, int phase, hipStream_t s, bool colour)
{
    if constexpr (seg_wide<N>() != seg_for<N>()) {
        static_assert(seg_wide<N>() == 4 * seg_for<N>(), "segments 4x, 2x and 1x of the narrowest");
        const int seg = pick_seg<N>(items, n);
        if (seg == seg_wide<N>()) return run_chunk_seg<N, T, seg_wide<N>()>(items, n, phase, s, colour);
        if (seg == 2 * seg_for<N>()) return run_chunk_seg<N, T, 2 * seg_for<N>()>(items, n, phase, s, colour);
    }
    return run_chunk_seg<N, T, seg_for<N>()>(items, n, phase, s, colour);
}

// DSS of node-major FP64 contributions ev ([n_local][5]) into q with M^-1
// and the wall projection, by the box finish kernel (one item)
template <int N, int SEG>
int32_t run_plain_finish_seg(const Mesh &m, const double *ev, double *q, hipStream_t s)
{
    Batch B{};
    B.n = 1;
    B.ca = 0.0;
    B.cb = 1.0;
    BatchItem &it = B.it[0];
    it.qout = q;
    it.Minv = stage_minv(m);  // the box filter's J w follows the metric mode
    it.nrm = m.dv.nrm;
    it.ev = (void *)ev;
    it.flag = nullptr;
    it.nu = (int)m.nu;
    it.nh = (int)m.nh;
    it.ni = (int)m.ni;
    it.nj = (int)m.nj;
    it.nz = m.d.ne[2];
    it.walls = m.walls ? 1 : 0;
    it.fx = fast_div((uint32_t)m.d.ne[0]);
    it.fy = fast_div((uint32_t)m.d.ne[1]);
    it.fseg = fast_div((uint32_t)(m.d.ne[0] / SEG));
    const int64_t mblk = (int64_t)(m.d.ne[0] / SEG) * m.d.ne[1] * m.d.ne[2];
    it.mblk = (int)mblk;
    it.ne = (int)m.ne;
    const int64_t bo = mblk + (m.walls ? (int64_t)(m.d.ne[0] / SEG) * m.d.ne[1] : 0);
    const int threads = ((SEG * N * N * N + 63) / 64) * 64;
    hipLaunchKernelGGL((k_fin_batch<N, SEG, double, true>), dim3((unsigned)bo), dim3(threads), 0, s, B);
    NUMA_HIP(hipGetLastError());
    return NUMA_OK;
}

template <int N>
int32_t run_plain_finish(const Mesh &m, const double *ev, double *q, hipStream_t s)
{
    StepItem it{};
    it.mesh = &m;
    if constexpr (seg_wide<N>() != seg_for<N>()) {
        const int seg = pick_seg<N>(&it, 1);
        if (seg == seg_wide<N>()) return run_plain_finish_seg<N, seg_wide<N>()>(m, ev, q, s);
        if (seg == 2 * seg_for<N>()) return run_plain_finish_seg<N, 2 * seg_for<N>()>(m, ev, q, s);
    }
    return run_plain_finish_seg<N, seg_for<N>()>(m, ev, q, s);
}

template <typename T>
int32_t run_stage_t(const StepItem *items, int n, int phase, hipStream_t s, bool colour)
{
    for (int c0 = 0; c0 < n; c0 += kMaxBatch) {
        const int c = n - c0 < kMaxBatch ? n - c0 : kMaxBatch;
        int32_t rc;
        switch (items[0].mesh->N) {
        case 1: rc = run_chunk<1, T>(items + c0, c, phase, s, colour); break;
        case 2: rc = run_chunk<2, T>(items + c0, c, phase, s, colour); break;
        case 3: rc = run_chunk<3, T>(items + c0, c, phase, s, colour); break;
        case 4: rc = run_chunk<4, T>(items + c0, c, phase, s, colour); break;
        case 5: rc = run_chunk<5, T>(items + c0, c, phase, s, colour); break;
        case 6: rc = run_chunk<6, T>(items + c0, c, phase, s, colour); break;
        case 7: rc = run_chunk<7, T>(items + c0, c, phase, s, colour); break;
        default: rc = run_chunk<8, T>(items + c0, c, phase, s, colour); break;
        }
        if (rc) return rc;
    }
    return NUMA_OK;
}

}  // namespace

bool box_batchable(const Mesh &m)
{
    if (m.d.kind != NUMA_MESH_BOX) return false;
    int seg;
    switch (m.N) {
    case 1: seg = seg_for<1>(); break;
    case 2: seg = seg_for<2>(); break;
    case 3: seg = seg_for<3>(); break;
    case 4: seg = seg_for<4>(); break;
    case 5: seg = seg_for<5>(); break;
    case 6: seg = seg_for<6>(); break;
    case 7: seg = seg_for<7>(); break;
    default: seg = seg_for<8>(); break;
    }
    return m.d.ne[0] % seg == 0;
}

int32_t launch_box_plain_finish(const Mesh &m, const double *ev, double *q, hipStream_t s)
{
    switch (m.N) {
    case 1: return run_plain_finish<1>(m, ev, q, s);
    case 2: return run_plain_finish<2>(m, ev, q, s);
    case 3: return run_plain_finish<3>(m, ev, q, s);
    case 4: return run_plain_finish<4>(m, ev, q, s);
    case 5: return run_plain_finish<5>(m, ev, q, s);
    case 6: return run_plain_finish<6>(m, ev, q, s);
    case 7: return run_plain_finish<7>(m, ev, q, s);
    default: return run_plain_finish<8>(m, ev, q, s);
    }
}

bool colour_ok(const Mesh &m)
{
    return m.stage_mode == NUMA_STAGE_COLOUR && m.d.kind == NUMA_MESH_BOX && m.metric_mode == NUMA_METRIC_RECOMPUTE &&
           m.N <= 4 && m.d.ne[0] % 2 == 0 && m.d.ne[1] % 2 == 0 && m.d.ne[2] % 2 == 0;
}

int32_t launch_batch_stage(const StepItem *items, int n, int32_t prec, int phase, hipStream_t s)
{
    // items the fused block kernels take (pencil.hip), the colour passes, the
    // rest; partitioned in chunks on the stack, with no host allocation
    constexpr int kChunk = 4 * kMaxBatch;
    StepItem part[3][kChunk];
    for (int c0 = 0; c0 < n; c0 += kChunk) {
        const int cn = n - c0 < kChunk ? n - c0 : kChunk;
        int cnt[3] = {0, 0, 0};
        for (int k = c0; k < c0 + cn; ++k) {
            const int g = pencil_stage_ok(items[k], prec) ? 0 : colour_ok(*items[k].mesh) ? 1 : 2;
            part[g][cnt[g]++] = items[k];
        }
        int32_t rc;
        if (cnt[0] && (rc = launch_pencil_stage(part[0], cnt[0], prec, phase, s))) return rc;
        for (int g = 1; g < 3; ++g) {
            if (!cnt[g]) continue;
            rc = prec == NUMA_PREC_MIXED ? run_stage_t<float>(part[g], cnt[g], phase, s, g == 1)
                                         : run_stage_t<double>(part[g], cnt[g], phase, s, g == 1);
            if (rc) return rc;
        }
    }
    return NUMA_OK;
}

}  // namespace numa
