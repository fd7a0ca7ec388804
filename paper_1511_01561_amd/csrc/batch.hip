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
    int mblk;             // finish blocks of the main layers: (nx/SEG) ny nz (split: of the face rows)
    FastDiv fx, fy, fseg;  // division by nx, ny and nx/SEG (colour passes: fseg by nx/2, fy by ny/2;
                           // split: fseg by ni)
    FastDiv frl;           // split: division by the face rows per element layer, nj + (N - 1) ny
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
// elements per workgroup of the split DSS (the run length along x): the column
// kernels' up to N = 4, above that as many as 256 lanes and an 80 KB tile
// (two workgroups per CU) hold: 7, 5, 4, 2 at N = 5..8
template <int N> constexpr int split_eb()
{
    constexpr int PP = (N + 1) * (N + 1), lanes = 256 / PP, lds = 2048 / (PP * (N + 1));
    return N <= 4 ? col_eb<N, double>() : (lanes < lds ? lanes : lds);
}
template <int N> constexpr int split_threads() { return ((split_eb<N>() * (N + 1) * (N + 1) + 63) / 64) * 64; }

template <int N, typename T, int MODE = 0>
constexpr int col_blocks() { return (sizeof(T) == 4 && N == 4) ? 4 : 1; }

// NUMA_STAGE_SPLIT: the DSS split between the element kernel and a finish
// kernel over the element faces.  The EB elements of a column workgroup are
// consecutive in the element order, so element q's west face (i = 0) and
// element q - 1's east face (i = N) are the same nodes whenever both lie in
// the workgroup and in one row (ex != 0): the workgroup adds those pairs in
// LDS.  A node whose (j, k) is interior to the element (0 < j, k < N) then has
// all its copies in the workgroup unless it sits on the x face that starts
// the run (q = 0 or ex = 0), and the element kernel finishes it itself: M^-1,
// the stage update and the state write (these nodes are never on a wall),
// except in the run's first element (see Fb).  What remains are the face
// nodes (gj or gk a multiple of N: 4N of the (N+1)^2 (j, k) pairs of an
// element, "face pairs") and the interior rows of a run's first element.
// Their contributions are written in two arrays:
//  * Fa [nz][ny][4N][ni][5] (of T): per element row (ey, ez), face pair fp and
//    lattice position gi = ex N + i (i < N) the five values of the
//    contribution of element ex at local i (at i = 0 the pair sum when the run
//    holds element ex - 1), so the finish reads each face row of the lattice
//    as one contiguous run per copy;
//  * Fb [ne][4N + (N-1)^2 (N+1)][5]: the copies the finish kernel takes at
//    run boundaries: slots 0..4N-1 the face pairs at i = N and 4N + ip the
//    interior pair ip at i = N of an element whose east neighbour is not in
//    its run; 4N + (N-1)^2 + ip N + i the interior pair ip at i < N of a run's
//    first element.  The finish kernel takes those N nodes of every interior
//    row at a run start together (whole 32-byte sectors of the state rows,
//    where single scattered nodes would cost a read-modify-write each), so
//    the element kernel finishes none of its first element's nodes.
// Fa, Fb and the face pairs fill (N+1)^3 values per element: the workspace's
// contribution scratch.
// Face pairs fp(j, k): k = 0: j; k = N: N + 1 + j; 0 < k < N: 2 (N+1) +
// 2 (k - 1) + (j == N).  Interior pairs: ip = (j - 1) + (N - 1)(k - 1).
template <int N>
__device__ __forceinline__ int split_fp(int j, int k)
{
    return k == 0 ? j : (k == N ? N + 1 + j : 2 * (N + 1) + 2 * (k - 1) + (j == N ? 1 : 0));
}
template <int N>
__device__ __forceinline__ void split_fp_jk(int fp, int &j, int &k)
{
    if (fp <= N) {
        j = fp;
        k = 0;
    } else if (fp < 2 * (N + 1)) {
        j = fp - (N + 1);
        k = N;
    } else {
        const int r = fp - 2 * (N + 1);
        k = 1 + (r >> 1);
        j = (r & 1) ? N : 0;
    }
}
template <int N> constexpr int split_nb() { return 4 * N + (N - 1) * (N - 1) * (N + 1); }

// what the split-DSS output of a column workgroup needs of its box item
struct SplitGeo {
    int nx, ny, nz, ni, nj, nu;
    FastDiv fx, fy;
};

// the run-interior nodes a lane of a column workgroup (EB elements, BT
// lanes) finishes: interior pair ip, element qq, local ii, not in the run's
// first element, whose west neighbour is not in the workgroup; I = -1 where
// the lane has no node in that pass
template <int N, int EB, int BT>
struct SplitPre {
    static constexpr int NIN = (N - 1) * (N - 1) * EB * N, SPL = NIN > 0 ? (NIN + BT - 1) / BT : 1;
    int32_t I[SPL];
    double m[SPL], qn[SPL][5];
};

// the lane's run-interior nodes and their M^-1 and q^n (loaded at the start
// of the kernel, used at its end)
template <int N, int EB, int BT>
__device__ __forceinline__ void split_prefetch(const BatchItem &it, const SplitGeo &gm, bool load_qn, int t, int e0,
                                               int new_, SplitPre<N, EB, BT> &pf)
{
    using S = SplitPre<N, EB, BT>;
#pragma unroll
    for (int p = 0; p < S::SPL; ++p) {
        pf.I[p] = -1;
        pf.m[p] = 0.0;
#pragma unroll
        for (int v = 0; v < 5; ++v) pf.qn[p][v] = 0.0;
    }
    if constexpr (S::NIN > 0) {
#pragma unroll
        for (int p = 0; p < S::SPL; ++p) {
            const int n = t + p * BT;
            if (n >= S::NIN) continue;
            const int ip = n / (EB * N), m = n - ip * (EB * N), qq = m / N, ii = m - qq * N;
            if (qq >= new_) continue;
            const BoxElem fe = box_elem((uint32_t)(e0 + qq), gm.fx, gm.fy);
            if (qq == 0 || fe.ex == 0) continue;  // a run's first element: the finish kernel takes it
            const int jj = 1 + ip % (N - 1), kk = 1 + ip / (N - 1);
            pf.I[p] = fe.ex * N + ii + gm.ni * (fe.ey * N + jj + gm.nj * (fe.ez * N + kk));
            pf.m[p] = it.Minv[pf.I[p]];
            if (load_qn)
#pragma unroll
                for (int v = 0; v < 5; ++v) pf.qn[p][v] = it.qn[pf.I[p] + v * gm.nu];
        }
    }
}

// after the contributions of the workgroup are in st ([q][l][5], synchronised):
// the copies the finish kernel takes at run boundaries (Fb), the face rows
// (Fa, the run's x pairs added) and the run-interior nodes (M^-1, the update
// sc, folded or not, the state)
template <int N, typename T, int EB, int BT>
__device__ __forceinline__ void split_store(const BatchItem &it, const SplitGeo &gm, const StageCoef &sc, bool fold,
                                            const T *st, int t, int e0, int new_, const SplitPre<N, EB, BT> &pf)
{
    constexpr int P = N + 1, NP = P * P * P, NFP = 4 * N, NIP = (N - 1) * (N - 1), NB = split_nb<N>();
    using S = SplitPre<N, EB, BT>;
    T *Fa = (T *)it.ev;
    // Fb: the east face (slot order: face pairs, then interior pairs) of an
    // element whose east neighbour is not in the run, the interior rows of a
    // run's first element (ip, then i); by the last wavefront where the face
    // rows below leave most of its lanes idle (N = 4: 8 of 64), else by all
    constexpr int RUN = EB * N * 5;  // values of one face pair of the workgroup
    constexpr bool LASTW = RUN <= BT - 48;
    constexpr int FBS = LASTW ? 64 : BT;
    T *Fb = Fa + 5 * (int64_t)gm.nz * gm.ny * NFP * gm.ni;
    const int tb = LASTW ? t - (BT - 64) : t;
    int ex = box_elem((uint32_t)e0, gm.fx, gm.fy).ex;  // x index of element qq, stepped along the run
    for (int qq = 0; tb >= 0 && qq < new_; ++qq, ex = ex + 1 == gm.nx ? 0 : ex + 1) {
        if (!(qq == EB - 1 || ex == gm.nx - 1 || qq == 0 || ex == 0)) continue;
        T *fb = Fb + (int64_t)(e0 + qq) * NB * 5;
        if (qq == EB - 1 || ex == gm.nx - 1) {
            for (int u = tb; u < (NFP + NIP) * 5; u += FBS) {
                const int slot = u / 5, v = u - slot * 5;
                int jj, kk;
                if (slot < NFP) {
                    split_fp_jk<N>(slot, jj, kk);
                } else {  // interior pairs (N > 1)
                    constexpr int M = N > 1 ? N - 1 : 1;
                    jj = 1 + (slot - NFP) % M;
                    kk = 1 + (slot - NFP) / M;
                }
                fb[u] = st[(qq * NP + N + P * (jj + P * kk)) * 5 + v];
            }
        }
        if (NIP > 0 && (qq == 0 || ex == 0)) {
            for (int u = tb; u < NIP * N * 5; u += FBS) {
                const int nd = u / 5, v = u - nd * 5, ip = nd / N, ii = nd - ip * N;
                const int jj = 1 + ip % (N - 1), kk = 1 + ip / (N - 1);
                fb[(NFP + NIP) * 5 + u] = st[(qq * NP + ii + P * (jj + P * kk)) * 5 + v];
            }
        }
    }
    // Fa: lane u < EB N 5 takes value v of node (qq, ii) of every face pair,
    // so that each store instruction writes one contiguous run of the pair's
    // row, and the lane's element, pair flag and offsets are formed once
    for (int u = t; u < RUN; u += BT) {
        const int nd = u / 5, v = u - nd * 5, qq = nd / N, ii = nd - qq * N;
        if (qq < new_) {
            const BoxElem fe = box_elem((uint32_t)(e0 + qq), gm.fx, gm.fy);
            const bool pair = ii == 0 && qq > 0 && fe.ex != 0;
            const T *s0 = st + (qq * NP + ii) * 5 + v, *s1 = st + ((qq - 1) * NP + N) * 5 + v;
            T *fo = Fa + (((int64_t)(fe.ez * gm.ny + fe.ey) * NFP) * gm.ni + fe.ex * N + ii) * 5 + v;
#pragma unroll
            for (int fp = 0; fp < NFP; ++fp) {
                int jj, kk;
                split_fp_jk<N>(fp, jj, kk);
                const int lo = P * (jj + P * kk) * 5;
                T val = s0[lo];
                if (pair) val += s1[lo];
                fo[(int64_t)fp * gm.ni * 5] = val;
            }
        }
    }
    if constexpr (S::NIN > 0) {
#pragma unroll
        for (int p = 0; p < S::SPL; ++p) {
            if (pf.I[p] < 0) continue;
            const int n = t + p * BT;
            const int ip = n / (EB * N), m = n - ip * (EB * N), qq = m / N, ii = m - qq * N;
            const int jj = 1 + ip % (N - 1), kk = 1 + ip / (N - 1);
            const int l = ii + P * (jj + P * kk), lw = N + P * (jj + P * kk);
            double r[5], o[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                r[v] = (double)st[(qq * NP + l) * 5 + v];
                if (ii == 0) r[v] += (double)st[((qq - 1) * NP + lw) * 5 + v];
                r[v] *= pf.m[p];
            }
            if (fold) {
#pragma unroll
                for (int v = 0; v < 5; ++v) o[v] = rk_update_folded(sc, pf.qn[p][v], r[v]);
            } else {
#pragma unroll
                for (int v = 0; v < 5; ++v)
                    o[v] = rk_update(sc, pf.qn[p][v], sc.b == 0.0 ? 0.0 : it.qs[pf.I[p] + v * gm.nu], r[v]);
            }
#pragma unroll
            for (int v = 0; v < 5; ++v) it.qout[pf.I[p] + v * gm.nu] = o[v];
            flag_nonfinite(it.flag, o, 5);
        }
    }
}

// MODE 0: write J w R node-major for the finish kernel (NUMA_STAGE_GATHER);
// MODE 1: one colour pass of NUMA_STAGE_COLOUR: the workgroup's elements are
// the elements of colour `colour` (parity of ex, ey, ez), EB consecutive ones
// along x, and every lane adds its nodes' J w R to the FP64 accumulator with
// a plain read-modify-write (no other element of the colour has the node).
// (NUMA_STAGE_SPLIT takes the two-pass k_elem_col2 below.)
template <int N, typename T, int MODE = 0>
__global__ __launch_bounds__((col_threads<N, T>()), (col_blocks<N, T, MODE>())) void k_elem_col(Batch B, int colour)
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

// The element kernel of the split DSS (NUMA_STAGE_SPLIT, above), with a
// two-pass tile.  k_elem_col keeps eight tile fields (8 (N+1)^3 doubles per
// element in FP64) and every field's zeta derivative in registers, which leaves
// room for two workgroups per CU.  Here the tile holds five fields at a time, the
// size of the output staging: first p', u, v, w, theta', from which the
// momentum and theta' rows of R follow (advection, pressure gradient,
// buoyancy), then rho u and rho v for the mass row (rho w enters it only
// through zeta, from the lane's own column).  The lane takes its column's
// values from the tile once per pass, the xi and eta rows per node.  Each term is
// the product and sum of k_elem_col (in mixed precision the tile and the
// contractions FP32, rho, 1/rho, rho'/rho and p' formed in FP64 as there);
// the tail is the split DSS.  FP64: three workgroups per CU at N = 4 (50 KB
// of LDS), four below (N = 3: 40 KB, a 16-byte stack frame, measured faster
// than three without it); N = 5..8 as noted below.  Mixed (N <= 4): four
// waves per SIMD.
template <int N, typename T> constexpr int col2_waves()
{
    return sizeof(T) == 4 ? 4 : (N <= 3 ? 4 : (N == 4 ? 3 : 2));
}
// doubles after each element's tile: at N = 4, 8 spread the xi and eta rows of
// the two or three elements a wavefront spans over the LDS banks (50,640
// bytes, still three workgroups per CU); at N = 3 the 40 KB tile has no room
template <int N, typename T = double> constexpr int col2_pad() { return sizeof(T) == 8 && N == 4 ? 8 : 0; }
// N = 5, 6 (seven and five elements per 256-lane workgroup, 60 and 69 KB of
// LDS): two waves per SIMD
template <int N, typename T = double>
__global__ __launch_bounds__((split_threads<N>()), (col2_waves<N, T>())) void k_elem_col2(Batch B)
{
    constexpr bool F64 = sizeof(T) == 8;
    constexpr int P = N + 1, PP = P * P, NP = PP * P, EB = split_eb<N>(), BT = split_threads<N>();
    constexpr int PAD = col2_pad<N, T>();
    __shared__ T s[EB][5 * NP + PAD];
    auto S = [&](int qq, int f, int l) -> T & { return s[qq][f * NP + l]; };
    const int g0 = (int)xcd_remap(blockIdx.x, gridDim.x) * EB;
    const BatchItem &it = B.it[batch_item(B, g0, false)];
    const RhsArgs<T> a = elem_args<T>(B, it);
    const int e0 = g0 - it.eoff;
    const int t = threadIdx.x, q = t / PP, c = t % PP, i = c % P, j = c / P;
    const bool act = q < EB && e0 + q < it.ne;
    const int new_ = it.ne - e0 < EB ? it.ne - e0 : EB;
    const SplitGeo gm{a.nx, a.ny, a.nz, a.ni, a.nj, (int)a.nu, a.fx, a.fy};
    const bool fold = B.fold != 0;
    const double cdt = it.cdt, gz = -a.g0;
    const int walls = it.walls;
    // per node of the column, formed in FP64 as in k_elem_col: rho, 1/rho and
    // rho' (FP64; in mixed precision rho'/rho, the buoyancy factor)
    double rho[P];
    T ir[P], bq[P];
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
            const double r_ = qp[0], u = qp[a.nu], v = qp[2 * a.nu], w = qp[3 * a.nu], tp = qp[4 * a.nu];
            const double rb = rf[0], tb = it.theta0, pb = rf[2 * a.nu];
            rho[k] = rb + r_;
            const double dl = r_ * tb + rb * tp + r_ * tp;
            const int l = c + PP * k;
            S(q, 0, l) = (T)(pb * eos_rel(dl / (rb * tb), a.gamma, a.eos));
            S(q, 1, l) = (T)u;
            S(q, 2, l) = (T)v;
            S(q, 3, l) = (T)w;
            S(q, 4, l) = (T)tp;
            const double ird = 1.0 / rho[k];
            ir[k] = (T)ird;
            bq[k] = F64 ? (T)r_ : (T)(r_ * ird);
        }
    }
    __syncthreads();  // first tile complete
    T res[P][5];
    T Di[P], Dj[P];
#pragma unroll
    for (int m = 0; m < P; ++m) {
        Di[m] = a.D[i * P + m];
        Dj[m] = a.D[j * P + m];
    }
    if (act) {
#pragma unroll
        for (int k = 0; k < P; ++k) {
            T mx[10];
            box_node_metric<T>(a.bm, ez, B.xi[k], c0 * B.w[k], c1, c2, c3, mx);
            const int l = c + PP * k;
            const T uu = S(q, 1, l), vv = S(q, 2, l), ww = S(q, 3, l), tt = S(q, 4, l);
            T dd[5][3];
#pragma unroll
            for (int f = 0; f < 5; ++f) {
                T da = 0, db = 0, dz = 0;
#pragma unroll
                for (int m = 0; m < P; ++m) {
                    da += Di[m] * S(q, f, m + P * (j + P * k));
                    db += Dj[m] * S(q, f, i + P * (m + P * k));
                    dz += a.D[k * P + m] * S(q, f, c + PP * m);
                }
                dd[f][0] = da;
                dd[f][1] = db;
                dd[f][2] = dz;
            }
            T Uc[3];
            Uc[0] = uu * mx[0];
            Uc[1] = vv * mx[4];
            Uc[2] = uu * mx[6] + vv * mx[7] + ww * mx[8];
            auto adv = [&](int f) -> T { return Uc[0] * dd[f][0] + Uc[1] * dd[f][1] + Uc[2] * dd[f][2]; };
            const T bk = F64 ? bq[k] * ir[k] : bq[k];
            T R[4];
            R[0] = -adv(1) - (dd[0][0] * mx[0] + dd[0][2] * mx[6]) * ir[k];
            R[1] = -adv(2) - (dd[0][1] * mx[4] + dd[0][2] * mx[7]) * ir[k];
            R[2] = -adv(3) - dd[0][2] * mx[8] * ir[k] + bk * gz;
            R[3] = -adv(4);
            const bool wall = walls && ((ez == 0 && k == 0) || (ez == a.nz - 1 && k == N));
            if (fold && !wall) {
                const T qv[4] = {uu, vv, ww, tt};
#pragma unroll
                for (int v = 0; v < 4; ++v) res[k][v + 1] = mx[9] * fma((T)cdt, R[v], qv[v]);
            } else {
#pragma unroll
                for (int v = 0; v < 4; ++v) res[k][v + 1] = mx[9] * R[v];
            }
        }
    }
    // the mass fluxes of the column, formed from the first tile: rho u and
    // rho v go through the second tile (their xi and eta rows), the column's
    // own values stay in registers for the zeta derivatives
    T fl[P][3];
    if (act) {
#pragma unroll
        for (int k = 0; k < P; ++k) {
            const int l = c + PP * k;
            fl[k][0] = (T)(rho[k] * (double)S(q, 1, l));
            fl[k][1] = (T)(rho[k] * (double)S(q, 2, l));
            fl[k][2] = (T)(rho[k] * (double)S(q, 3, l));
        }
    }
    __syncthreads();  // first tile read
    if (act) {
#pragma unroll
        for (int k = 0; k < P; ++k)
#pragma unroll
            for (int f = 0; f < 2; ++f) S(q, f, c + PP * k) = fl[k][f];
    }
    __syncthreads();  // second tile complete
    if (act) {
#pragma unroll
        for (int k = 0; k < P; ++k) {
            T mx[10];
            box_node_metric<T>(a.bm, ez, B.xi[k], c0 * B.w[k], c1, c2, c3, mx);
            T da = 0, db = 0, dz[3] = {0, 0, 0};
#pragma unroll
            for (int m = 0; m < P; ++m) {
                da += Di[m] * S(q, 0, m + P * (j + P * k));
                db += Dj[m] * S(q, 1, i + P * (m + P * k));
#pragma unroll
                for (int f = 0; f < 3; ++f) dz[f] += a.D[k * P + m] * fl[m][f];
            }
            const T R0 = -((da * mx[0] + dz[0] * mx[6]) + (db * mx[4] + dz[1] * mx[7]) + dz[2] * mx[8]);
            const bool wall = walls && ((ez == 0 && k == 0) || (ez == a.nz - 1 && k == N));
            res[k][0] = (fold && !wall) ? mx[9] * fma((T)cdt, R0, bq[k]) : mx[9] * R0;
        }
    }
    // the run-interior nodes' M^-1 and q^n (issued here, where the tiles'
    // registers are free)
    SplitPre<N, EB, BT> pf;
    split_prefetch<N, EB, BT>(it, gm, B.ca != 0.0, t, e0, new_, pf);
    __syncthreads();  // second tile read
    T *st = &s[0][0];
    if (act) {
#pragma unroll
        for (int k = 0; k < P; ++k)
#pragma unroll
            for (int v = 0; v < 5; ++v) st[(q * NP + c + PP * k) * 5 + v] = res[k][v];
    }
    __syncthreads();
    split_store<N, T, EB, BT>(it, gm, StageCoef{B.ca, B.cb, cdt}, fold, st, t, e0, new_, pf);
}

// NUMA_STAGE_SPLIT finish: the face nodes and the run-start interior nodes.
// mblk blocks of an item take the face rows of the lattice, one node per
// lane along x: per element layer ez the level gk = ez N (all nj rows), then
// the levels ez N + 1 .. ez N + N - 1 (the ny rows gj = ey N), and with walls
// the top level gk = nz N; frl divides by the rows per layer
// nj + (N - 1) ny (fseg divides by ni).  The other blocks (interleaved) take
// the interior rows of a run's first element, N nodes per row (i < N): the
// elements e = c EB (one per element workgroup), then the row starts
// e = r nx that are not multiples of EB.  Every node's
// copies are read in a fixed order (z copies, y copies, then the x copies of
// each), summed in FP64, multiplied by M^-1, projected at the walls and
// advanced by the stage update (PLAIN: the summed value itself, for the
// filter: the stage operands are not read).
template <int N, typename T, bool PLAIN = false>
__global__ __launch_bounds__(256) void k_fin_split(Batch B)
{
    constexpr int NFP = 4 * N, NIP = (N - 1) * (N - 1), NB = split_nb<N>(), EB = split_eb<N>();
    const int g = (int)xcd_remap(blockIdx.x, gridDim.x);
    const BatchItem &it = B.it[batch_item(B, g, true)];
    const int nx = (int)it.fx.d, ny = (int)it.fy.d, nz = it.nz, ni = it.ni, nj = it.nj;
    // the item's blocks: mblk face-row blocks and nbb run-start blocks, the
    // latter spread evenly (block k at k S + S - 1, S = total / nbb), so that
    // every XCD's range of the launch holds its share of the scattered ones
    int lb = g - it.boff;
    const int nbb = NIP == 0 ? 0 : (((it.ne + EB - 1) / EB + ny * nz) * NIP * N + 255) / 256;
    bool runstart = false;
    if (NIP > 0 && nbb > 0) {
        const int S = (it.mblk + nbb) / (NIP > 0 ? nbb : 1);
        if (lb < nbb * S) {
            const int k = lb / S;
            runstart = lb - k * S == S - 1;
            lb = runstart ? k : lb - k;
        } else {
            lb -= nbb;
        }
    }
    const int64_t vs = (int64_t)nz * ny * NFP * ni;
    const T *Fa = (const T *)it.ev, *Fb = Fa + 5 * vs;
    int gi, gj, gk;
    double r[5] = {0, 0, 0, 0, 0};
    // the stage update's operands are loaded as soon as the node is known,
    // before its copies: one memory round trip per node instead of two
    const StageCoef sc{B.ca, B.cb, it.cdt};
    double mi, qnv[5], qsv[5];
    int32_t I;
    bool folded;
    auto update_loads = [&]() {
        I = gi + ni * (gj + nj * gk);
        folded = !PLAIN && B.fold && !(it.walls && (gk == 0 || gk == nz * N));
        mi = it.Minv[I];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            qnv[v] = PLAIN || sc.a == 0.0 ? 0.0 : it.qn[I + v * it.nu];
            qsv[v] = PLAIN || folded || sc.b == 0.0 ? 0.0 : it.qs[I + v * it.nu];
        }
    };
    if (!runstart) {
        const int rl = (int)it.frl.d;
        const int nrows = nz * rl + (it.walls ? nj : 0);
        const uint32_t id = (uint32_t)lb * 256u + threadIdx.x;
        if (id >= (uint32_t)nrows * (uint32_t)ni) return;
        const uint32_t R = fdiv(id, it.fseg);
        gi = (int)(id - R * (uint32_t)ni);
        const uint32_t ezr = fdiv(R, it.frl);
        int rr = (int)(R - ezr * (uint32_t)rl);
        if ((int)ezr == nz) {  // the top wall level
            gk = nz * N;
            gj = rr;
        } else if (rr < nj) {
            gk = (int)ezr * N;
            gj = rr;
        } else {
            rr -= nj;
            const uint32_t kk = fdiv((uint32_t)rr, it.fy);
            gj = (rr - (int)kk * ny) * N;
            gk = (int)ezr * N + 1 + (int)kk;
        }
        update_loads();
        // copies: z (element layer, local k), y (element row, local j)
        int zc[2], kc[2], nzc = 1, yc[2], jc[2], nyc = 1;
        zc[0] = gk / N;
        kc[0] = gk % N;
        zc[1] = zc[0];
        kc[1] = kc[0];
        if (kc[0] == 0) {
            if (it.walls && gk == nz * N) {
                zc[0] = nz - 1;
                kc[0] = N;
            } else if (!(it.walls && gk == 0)) {
                zc[1] = zc[0] == 0 ? nz - 1 : zc[0] - 1;
                kc[1] = N;
                nzc = 2;
            }
        }
        yc[0] = gj / N;
        jc[0] = gj % N;
        yc[1] = yc[0];
        jc[1] = jc[0];
        if (jc[0] == 0) {
            yc[1] = yc[0] == 0 ? ny - 1 : yc[0] - 1;
            jc[1] = N;
            nyc = 2;
        }
        const int ex = gi / N;
        const bool xface = gi % N == 0;
        // the face rows' copies (absent ones are not loaded) are loaded
        // together, then summed; the run-start x copies (Fb, at most one
        // node in EB N of a row) after them
        T ca[2][2][5];
#pragma unroll
        for (int z = 0; z < 2; ++z)
#pragma unroll
            for (int y = 0; y < 2; ++y) {
                const bool has = z < nzc && y < nyc;
                const int64_t o = ((int64_t)(zc[z] * ny + yc[y]) * NFP + split_fp<N>(jc[y], kc[z])) * ni + gi;
#pragma unroll
                for (int v = 0; v < 5; ++v) ca[z][y][v] = has ? Fa[o * 5 + v] : (T)0;
            }
#pragma unroll
        for (int z = 0; z < 2; ++z)
#pragma unroll
            for (int y = 0; y < 2; ++y)
                if (z < nzc && y < nyc)
#pragma unroll
                    for (int v = 0; v < 5; ++v) r[v] += (double)ca[z][y][v];
        if (xface) {
#pragma unroll
            for (int z = 0; z < 2; ++z)
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                    const int ec = ex + nx * (yc[y] + ny * zc[z]);
                    if (z < nzc && y < nyc && (ex == 0 || ec % EB == 0)) {
                        const int64_t ob = ((int64_t)(ex == 0 ? ec + nx - 1 : ec - 1) * NB + split_fp<N>(jc[y], kc[z])) * 5;
#pragma unroll
                        for (int v = 0; v < 5; ++v) r[v] += (double)Fb[ob + v];
                    }
                }
        }
    } else {
        if constexpr (NIP == 0) {
            return;
        } else {
            const int nwg = (it.ne + EB - 1) / EB, nrs = ny * nz;
            const int id = lb * 256 + (int)threadIdx.x;
            const int cand = id / (NIP * N), rr = id - cand * (NIP * N), ip = rr / N, i = rr - ip * N;
            if (cand >= nwg + nrs) return;
            int e;
            if (cand < nwg) {
                e = cand * EB;
            } else {
                e = (cand - nwg) * nx;
                if (e % EB == 0) return;  // a workgroup start: taken above
            }
            const BoxElem be = box_elem((uint32_t)e, it.fx, it.fy);
            const int jj = 1 + ip % (N - 1), kk = 1 + ip / (N - 1);
            gi = be.ex * N + i;
            gj = be.ey * N + jj;
            gk = be.ez * N + kk;
            update_loads();
            const int ew = be.ex == 0 ? e + nx - 1 : e - 1;  // the element west of the run start
            const int64_t o0 = ((int64_t)e * NB + NFP + NIP + ip * N + i) * 5, o1 = ((int64_t)ew * NB + NFP + ip) * 5;
            T c0[5], c1[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                c0[v] = Fb[o0 + v];
                c1[v] = i == 0 ? Fb[o1 + v] : (T)0;
            }
#pragma unroll
            for (int v = 0; v < 5; ++v) r[v] = i == 0 ? (double)c0[v] + (double)c1[v] : (double)c0[v];
        }
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) r[v] *= mi;
    double o[5];
    if (folded) {
#pragma unroll
        for (int v = 0; v < 5; ++v) o[v] = rk_update_folded(sc, qnv[v], r[v]);
    } else {
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
        for (int v = 0; v < 5; ++v) o[v] = rk_update(sc, qnv[v], qsv[v], r[v]);
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) it.qout[I + v * it.nu] = o[v];
    flag_nonfinite(it.flag, o, 5);
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

// The Boyd-Vandeven filter of a box with the recomputed metric through the
// split DSS: the column workgroup of the stage (EB consecutive elements, a lane
// per (i, j) column) gathers the state into an LDS tile, applies F along xi
// and eta through the tile and along zeta in the lane's registers (the same
// fma chains in the same direction order as k_filter), weights by J w and
// hands J w (F q) to the split DSS: the run-interior nodes are finished here
// (M^-1, no stage update), the others by k_fin_split.  The state is filtered
// in place: the nodes finished here are read by no other workgroup, and the
// face kernel reads only the contributions.
struct FilterSplit {
    BatchItem it;             // qs: the state read, qout: the state written (the same array)
    double w[kMaxP];          // GLL weights
    double F[kMaxP * kMaxP];  // 1D nodal filter matrix F[i * (N+1) + m]
};

template <int N>
__global__ __launch_bounds__((split_threads<N>())) void k_filter_col(FilterSplit A)
{
    constexpr int P = N + 1, PP = P * P, NP = PP * P, EB = split_eb<N>(), BT = split_threads<N>();
    constexpr int PAD = col2_pad<N, double>();  // the two-pass stage kernel's bank spread
    __shared__ double s[EB][5 * NP + PAD];
    auto S = [&](int qq, int f, int l) -> double & { return s[qq][f * NP + l]; };
    // the 1D filter matrix: in LDS up to N = 4; above, the lane's xi and eta
    // rows in registers and the zeta row from the kernel arguments, so that
    // the N = 7 tile (80 KB) leaves room for two workgroups per CU
    constexpr bool FREG = N >= 5;
    __shared__ double Fs[FREG ? 1 : PP];
    double Fi[P], Fj[P];
#pragma unroll
    for (int m = 0; m < P; ++m) {
        Fi[m] = FREG ? A.F[((int)threadIdx.x % PP % P) * P + m] : 0.0;
        Fj[m] = FREG ? A.F[((int)threadIdx.x % PP / P) * P + m] : 0.0;
    }
    const BatchItem &it = A.it;
    const int e0 = (int)xcd_remap(blockIdx.x, gridDim.x) * EB;
    const int t = threadIdx.x, q = t / PP, c = t % PP, i = c % P, j = c / P;
    const bool act = q < EB && e0 + q < it.ne;
    if (!FREG && t < PP) Fs[t] = A.F[t];
    const int new_ = it.ne - e0 < EB ? it.ne - e0 : EB;
    const SplitGeo gm{(int)it.fx.d, (int)it.fy.d, it.nz, it.ni, it.nj, it.nu, it.fx, it.fy};
    SplitPre<N, EB, BT> pf;
    split_prefetch<N, EB, BT>(it, gm, false, t, e0, new_, pf);
    double jw[P];
    if (act) {
        const BoxElem be = box_elem((uint32_t)(e0 + q), it.fx, it.fy);
        const double c0 = it.hcol[(int64_t)(be.ex + gm.nx * be.ey) * (4 * PP) + c];
        int gi = be.ex * N + i, gj = be.ey * N + j;
        if (gi == gm.ni) gi = 0;
        if (gj == gm.nj) gj = 0;
        const int base = gi + gm.ni * gj, layer = gm.ni * gm.nj;
#pragma unroll
        for (int k = 0; k < P; ++k) {
            int gk = be.ez * N + k;
            if (gk == it.nkw) gk = 0;
            const int32_t I = base + layer * gk;
#pragma unroll
            for (int v = 0; v < 5; ++v) S(q, v, c + PP * k) = it.qs[I + v * gm.nu];
            jw[k] = c0 * A.w[k];
        }
    }
    __syncthreads();
    double x[5][P];
    if (act) {  // xi
#pragma unroll
        for (int k = 0; k < P; ++k)
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                double r = 0.0;
#pragma unroll
                for (int m = 0; m < P; ++m) r = fma(FREG ? Fi[m] : Fs[i * P + m], S(q, v, m + P * (j + P * k)), r);
                x[v][k] = r;
            }
    }
    __syncthreads();
    if (act)
#pragma unroll
        for (int k = 0; k < P; ++k)
#pragma unroll
            for (int v = 0; v < 5; ++v) S(q, v, c + PP * k) = x[v][k];
    __syncthreads();
    double res[P][5];
    if (act) {  // eta through the tile, zeta in registers, times J w
#pragma unroll
        for (int k = 0; k < P; ++k)
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                double r = 0.0;
#pragma unroll
                for (int m = 0; m < P; ++m) r = fma(FREG ? Fj[m] : Fs[j * P + m], S(q, v, i + P * (m + P * k)), r);
                x[v][k] = r;
            }
#pragma unroll
        for (int k = 0; k < P; ++k)
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                double r = 0.0;
#pragma unroll
                for (int m = 0; m < P; ++m) r = fma(FREG ? A.F[k * P + m] : Fs[k * P + m], x[v][m], r);
                res[k][v] = jw[k] * r;
            }
    }
    __syncthreads();  // tile read
    double *st = &s[0][0];
    if (act)
#pragma unroll
        for (int k = 0; k < P; ++k)
#pragma unroll
            for (int v = 0; v < 5; ++v) st[(q * NP + c + PP * k) * 5 + v] = res[k][v];
    __syncthreads();
    split_store<N, double, EB, BT>(it, gm, StageCoef{0.0, 0.0, 1.0}, false, st, t, e0, new_, pf);
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

// the fields of a batch item that the split finish (k_fin_split) reads, for
// the column workgroups of EB elements; returns the item's finish blocks
int64_t split_item(const Mesh &m, int eb, BatchItem &it)
{
    const int N = m.N, ny = m.d.ne[1], nz = m.d.ne[2];
    const int64_t rl = m.nj + (int64_t)(N - 1) * ny;
    const int64_t rows = nz * rl + (m.walls ? m.nj : 0);
    const int64_t nwg = (m.ne + eb - 1) / eb;
    it.fseg = fast_div((uint32_t)m.ni);
    it.frl = fast_div((uint32_t)rl);
    it.mblk = (int)((rows * m.ni + 255) / 256);
    return it.mblk + ((nwg + (int64_t)ny * nz) * ((int64_t)(N - 1) * (N - 1) * N) + 255) / 256;
}

template <int N, typename T, int SEG>
int32_t run_chunk_seg(const StepItem *items, int n, int phase, hipStream_t s, int mode)
{
    const bool colour = mode == 1, split = mode == 2;
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
    const int eb = split ? split_eb<N>() : col ? col_eb<N, T>() : 1;
    // FP64 update that uses q_s (b != 0): the column and one-node-per-lane
    // element kernels fold q_s into the contributions (the streaming one,
    // which runs at its register limit, does not)
    B.fold = (std::is_same<T, double>::value && B.cb != 0.0 && (split || !(recompute && kind == 1))) ? 1 : 0;
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
        // the gather finish's segments (a split item's x extent need not hold
        // one: its fields are set below)
        const int nseg = m.d.ne[0] / SEG > 0 ? m.d.ne[0] / SEG : 1;
        it.fseg = fast_div((uint32_t)nseg);
        const int64_t mblk = (int64_t)nseg * m.d.ne[1] * m.d.ne[2];
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
        } else if (split) {  // face rows, 256 lattice points per block, then the run starts
            eo += (m.ne + eb - 1) / eb * eb;
            bo += split_item(m, eb, it);
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
    if (split) {
        if constexpr (kind == 0) {
            if (phase == 0) {
                hipLaunchKernelGGL((k_elem_col2<N, T>), dim3((unsigned)(eo / eb)), dim3(split_threads<N>()), 0, s, B);
            } else {
                hipLaunchKernelGGL((k_fin_split<N, T>), dim3((unsigned)bo), dim3(256), 0, s, B);
            }
            NUMA_HIP(hipGetLastError());
            return NUMA_OK;
        } else if constexpr (std::is_same<T, double>::value) {
            if (phase == 0)
                hipLaunchKernelGGL((k_elem_col2<N>), dim3((unsigned)(eo / eb)), dim3(split_threads<N>()), 0, s, B);
            else
                hipLaunchKernelGGL((k_fin_split<N, T>), dim3((unsigned)bo), dim3(256), 0, s, B);
            NUMA_HIP(hipGetLastError());
            return NUMA_OK;
        }
        set_error("split DSS: no element kernel for this order and precision");
        return NUMA_EUNSUPPORTED;
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
int32_t run_chunk(const StepItem *items, int n, int phase, hipStream_t s, int mode)
{
    if constexpr (seg_wide<N>() != seg_for<N>()) {
        static_assert(seg_wide<N>() == 4 * seg_for<N>(), "segments 4x, 2x and 1x of the narrowest");
        const int seg = pick_seg<N>(items, n);
        if (seg == seg_wide<N>()) return run_chunk_seg<N, T, seg_wide<N>()>(items, n, phase, s, mode);
        if (seg == 2 * seg_for<N>()) return run_chunk_seg<N, T, 2 * seg_for<N>()>(items, n, phase, s, mode);
    }
    return run_chunk_seg<N, T, seg_for<N>()>(items, n, phase, s, mode);
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
int32_t run_stage_t(const StepItem *items, int n, int phase, hipStream_t s, int mode)
{
    for (int c0 = 0; c0 < n; c0 += kMaxBatch) {
        const int c = n - c0 < kMaxBatch ? n - c0 : kMaxBatch;
        int32_t rc;
        switch (items[0].mesh->N) {
        case 1: rc = run_chunk<1, T>(items + c0, c, phase, s, mode); break;
        case 2: rc = run_chunk<2, T>(items + c0, c, phase, s, mode); break;
        case 3: rc = run_chunk<3, T>(items + c0, c, phase, s, mode); break;
        case 4: rc = run_chunk<4, T>(items + c0, c, phase, s, mode); break;
        case 5: rc = run_chunk<5, T>(items + c0, c, phase, s, mode); break;
        case 6: rc = run_chunk<6, T>(items + c0, c, phase, s, mode); break;
        case 7: rc = run_chunk<7, T>(items + c0, c, phase, s, mode); break;
        default: rc = run_chunk<8, T>(items + c0, c, phase, s, mode); break;
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

namespace {

template <int N>
int32_t run_filter_split(const Mesh &m, const double *F, double *q, hipStream_t s)
{
    constexpr int EB = split_eb<N>();
    FilterSplit A{};
    BatchItem &it = A.it;
    it.qs = q;
    it.qout = q;
    it.qn = nullptr;
    it.Minv = stage_minv(m);
    it.nrm = m.dv.nrm;
    it.ev = m.dv.ev64;
    it.hcol = m.dv.hcol;
    it.flag = nullptr;
    it.nu = (int)m.nu;
    it.nh = (int)m.nh;
    it.ni = (int)m.ni;
    it.nj = (int)m.nj;
    it.nkw = m.d.periodic[2] ? (int)m.nk : -1;
    it.nz = m.d.ne[2];
    it.walls = m.walls ? 1 : 0;
    it.ne = (int)m.ne;
    it.fx = fast_div((uint32_t)m.d.ne[0]);
    it.fy = fast_div((uint32_t)m.d.ne[1]);
    it.cdt = 1.0;
    it.eoff = 0;
    it.boff = 0;
    const int64_t bo = split_item(m, EB, it);
    for (int k = 0; k <= N; ++k) A.w[k] = m.w[k];
    for (int k = 0; k < (N + 1) * (N + 1); ++k) A.F[k] = F[k];
    hipLaunchKernelGGL((k_filter_col<N>), dim3((unsigned)((m.ne + EB - 1) / EB)), dim3(split_threads<N>()), 0, s, A);
    // the face nodes: the split finish with the identity update (a = b = 0, cdt = 1)
    Batch B{};
    B.n = 1;
    B.fold = 0;
    B.ca = 0.0;
    B.cb = 0.0;
    B.it[0] = it;
    hipLaunchKernelGGL((k_fin_split<N, double, true>), dim3((unsigned)bo), dim3(256), 0, s, B);
    NUMA_HIP(hipGetLastError());
    return NUMA_OK;
}

}  // namespace

bool filter_split_ok(const Mesh &m)
{
    return split_ok(m, NUMA_PREC_FP64);
}

int32_t launch_filter_split(const Mesh &m, const double *F, double *q, hipStream_t s)
{
    switch (m.N) {
    case 1: return run_filter_split<1>(m, F, q, s);
    case 2: return run_filter_split<2>(m, F, q, s);
    case 3: return run_filter_split<3>(m, F, q, s);
    case 4: return run_filter_split<4>(m, F, q, s);
    case 5: return run_filter_split<5>(m, F, q, s);
    case 6: return run_filter_split<6>(m, F, q, s);
    case 7: return run_filter_split<7>(m, F, q, s);
    case 8: return run_filter_split<8>(m, F, q, s);
    default:
        set_error("filter: the split DSS takes N <= 8");
        return NUMA_EUNSUPPORTED;
    }
}

bool colour_ok(const Mesh &m)
{
    return m.stage_mode == NUMA_STAGE_COLOUR && m.d.kind == NUMA_MESH_BOX && m.metric_mode == NUMA_METRIC_RECOMPUTE &&
           m.N <= 4 && m.d.ne[0] % 2 == 0 && m.d.ne[1] % 2 == 0 && m.d.ne[2] % 2 == 0;
}

// NUMA_STAGE_SPLIT runs a column element kernel (recomputed metric; N <= 4,
// and in FP64 N = 5, 6 with the two-pass kernel); its finish takes any x
// extent.  NUMA_STAGE_AUTO takes it in FP64 (measured faster than the gather
// there; in mixed precision the gather, whose FP32 contributions are half the
// bytes, is faster)
bool split_ok(const Mesh &m, int32_t prec)
{
    const bool mode = m.stage_mode == NUMA_STAGE_SPLIT || (m.stage_mode == NUMA_STAGE_AUTO && prec == NUMA_PREC_FP64);
    const int nmax = prec == NUMA_PREC_FP64 ? 8 : 4;
    return mode && m.d.kind == NUMA_MESH_BOX && m.metric_mode == NUMA_METRIC_RECOMPUTE && m.N <= nmax;
}

int32_t launch_batch_stage(const StepItem *items, int n, int32_t prec, int phase, hipStream_t s)
{
    // items the fused block kernels take (pencil.hip), the colour passes, the
    // split DSS, the rest; partitioned in chunks on the stack, with no host
    // allocation
    constexpr int kChunk = 4 * kMaxBatch;
    StepItem part[4][kChunk];
    for (int c0 = 0; c0 < n; c0 += kChunk) {
        const int cn = n - c0 < kChunk ? n - c0 : kChunk;
        int cnt[4] = {0, 0, 0, 0};
        for (int k = c0; k < c0 + cn; ++k) {
            const Mesh &m = *items[k].mesh;
            const int g = pencil_stage_ok(items[k], prec) ? 0 : colour_ok(m) ? 1 : split_ok(m, prec) ? 2 : 3;
            if (g == 3 && !box_batchable(m)) {
                set_error("batched stage: a box mesh whose x element count does not fit the finish segment");
                return NUMA_EUNSUPPORTED;
            }
            part[g][cnt[g]++] = items[k];
        }
        int32_t rc;
        if (cnt[0] && (rc = launch_pencil_stage(part[0], cnt[0], prec, phase, s))) return rc;
        for (int g = 1; g < 4; ++g) {
            if (!cnt[g]) continue;
            const int mode = g == 1 ? 1 : g == 2 ? 2 : 0;
            rc = prec == NUMA_PREC_MIXED ? run_stage_t<float>(part[g], cnt[g], phase, s, mode)
                                         : run_stage_t<double>(part[g], cnt[g], phase, s, mode);
            if (rc) return rc;
        }
    }
    return NUMA_OK;
}

}  // namespace numa
