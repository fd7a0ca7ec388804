// Fused stage on box meshes: the element right-hand side, the direct
// stiffness summation, M^-1, the wall projection and the stage update in one
// kernel per block of element columns, plus a small kernel for the nodes the
// blocks share.
//
// A workgroup owns a block of TX x TY element columns and TZ element layers
// and walks its layers from the bottom up.  Per layer it gathers the state
// of its elements, differentiates them (the column scheme of k_elem_col: a
// lane per (i, j) column of an element, zeta contractions from registers, xi
// and eta through the LDS tile), and stages the contributions J w R of all
// its element-local nodes in LDS.  A second set of lanes then sums, per
// lattice column of the block, the copies of each node in LDS (the DSS inside
// the block: one workgroup owns all the copies, so the sum needs neither
// atomics nor a colouring), carries the top level's partial sum to the next
// layer, and finishes every node whose copies all lie in the block: multiply
// by M^-1, project at the walls, apply the stage update and write the state.
// This replaces the round trip of the element-local contributions through
// HBM of the two-kernel stage (k_elem_col + k_fin_batch).
//
// Shared nodes.  x: the block owns the lattice columns gi in
// [bx WX, (bx + 1) WX) and recomputes the contribution of the western
// neighbour element at its east face (i = N) itself: a halo of one element
// column whose xi derivatives need the neighbour's nodes, while the eta and
// zeta derivatives on the shared face are the block's own.  So no node on an
// x block boundary is shared between workgroups, and every state row a block
// writes is one aligned run of WX nodes.  y and z: the nodes on a block's
// y faces (and on its z faces between blocks) are written as partial sums to
// a scratch array; k_pencil_seam adds the two (or four) partial sums of each
// such node in a fixed order and finishes it.  Every sum is taken in a fixed
// order, so results are deterministic and a mesh's result does not depend on
// what it is batched with.
//
// Requirements (pencil_ok): box with no-flux walls in z, recomputed metric,
// N in 2..4, nx a multiple of TX, ny of TY, the stage's input and output
// states distinct (a block writes finished nodes while others still gather).
#include "kernels.h"

namespace numa {
namespace {

using namespace dev;

constexpr int kMaxPenBatch = 16;

// block shape: element columns per block (the main lanes, one per element
// column (i, j), fill four wavefronts at N = 4, five at N = 3 (with the halo
// wavefront), three at N = 2) and lanes for the halo element
template <int N> constexpr int pen_tx() { return N == 4 ? 4 : 8; }
template <int N> constexpr int pen_ty() { return 2; }
template <int N> constexpr int pen_main() { return pen_tx<N>() * pen_ty<N>() * (N + 1) * (N + 1); }
// the halo lanes: at least one per node of the halo faces (TY (N+1)^2)
template <int N> constexpr int pen_threads()
{
    return ((pen_main<N>() + pen_ty<N>() * (N + 1) * (N + 1) + 63) / 64) * 64;
}
constexpr int kSeamThreads = 256;

struct PenItem {
    const double *qs;  // stage input state [5][nu]
    double *qout;      // stage output state (distinct from qs)
    const double *qn;  // reference state of the stage update
    const double *ref, *Minv, *nrm, *hcol;
    double *py;        // partial sums on the y block faces [nby][2][nbz][WZ+1][ni][5]
    double *pz;        // partial sums on the z block faces [nbz][2][nj][ni][5]
    int32_t *flag;     // non-finite flag of the item's state, or null
    int64_t nu, nh;
    int ni, nj, nk;    // lattice extents (nk = nz N + 1 levels)
    int nx, ny, nz;
    int nbx, nby, nbz, tz;  // blocks along x, y, z; element layers per block
    FastDiv fbx, fby;
    int boff;          // first block of this item in the launch
    int soff;          // first seam workgroup of this item in the launch
    int srows, sblk;   // seam rows; workgroups per row
    double cdt, theta0;
    BoxMetric bm;
};

struct PenBatch {
    int n;
    int fold;  // FP64 stages that use q_s: contributions J w (q_s + cdt R) away from the walls
    double ca, cb;
    double gamma, g0;
    const void *D;
    const double *xi, *w;
    double eos[kEosTerms];
    PenItem it[kMaxPenBatch];
};
static_assert(sizeof(PenBatch) <= 4096, "the batch table must fit the kernel arguments");

__device__ __forceinline__ int pen_item(const PenBatch &B, int g, bool seam)
{
    int k = 0;
    while (k + 1 < B.n && g >= (seam ? B.it[k + 1].soff : B.it[k + 1].boff)) ++k;
    return k;
}

// M^-1, wall projection and stage update of unique node I from the summed
// contributions r (as box_finish_node)
__device__ __forceinline__ void pen_finish(const PenItem &it, const PenBatch &B, int32_t I, double *r, bool wall)
{
    const StageCoef sc{B.ca, B.cb, it.cdt};
    const double mi = it.Minv[I];
    double qnv[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) qnv[v] = sc.a == 0.0 ? 0.0 : it.qn[I + v * it.nu];
#pragma unroll
    for (int v = 0; v < 5; ++v) r[v] *= mi;
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
    p.walls = 1;
    noflux(p, I, r[1], r[2], r[3]);
#pragma unroll
    for (int v = 0; v < 5; ++v) it.qout[I + v * it.nu] = o[v] = rk_update(sc, qnv[v], it.qs[I + v * it.nu], r[v]);
    flag_nonfinite(it.flag, o, 5);
}

// workgroups per CU the block kernel is compiled for: two at N = 4 (the
// FP64 tile and halo take 75 KB of LDS), otherwise as the registers allow
template <int N, typename T>
constexpr int pen_min_blocks() { return N == 4 ? 2 : 1; }

// The state and reference values a lane gathers for one layer: main lanes
// the N+1 nodes of their column, halo lanes up to N+1 halo nodes.
constexpr int kGather = 7;  // rho', u, v, w, theta', rho_bar, p_bar

template <int N, typename T>
__global__ __launch_bounds__(pen_threads<N>(), (pen_min_blocks<N, T>())) void k_pencil(PenBatch B)
{
    constexpr int P = N + 1, PP = P * P, NP = PP * P;
    constexpr int TX = pen_tx<N>(), TY = pen_ty<N>(), NE = TX * TY, ML = pen_main<N>();
    constexpr int BT = pen_threads<N>(), HL = BT - ML, WX = TX * N, WY = TY * N;
    constexpr int HN = TY * N * PP;  // halo nodes with m < N per layer
    constexpr bool F64 = sizeof(T) == 8;
    static_assert(HL >= TY * PP, "one halo lane per halo face node");
    static_assert((HN + HL - 1) / HL <= P, "a halo lane gathers at most N+1 nodes");
    static_assert(WX * (WY + 1) <= ML, "the summing lanes are main lanes");
    // element tile (7 fields: rho u, rho v, u, v, w, theta', p'); after the
    // derivatives the same memory holds the contributions [NE][P][PP][5]
    __shared__ T s[NE][7][NP];
    // halo: fields rho u, u, v, w, theta', p' of the western neighbour
    // elements at local (m, j, k), m = 0..N (m = N: the block's own face)
    __shared__ T ht[TY][6][NP];
    // the block's west face (i = 0 of qx = 0): rho w, rho v, 1/rho, buoyancy
    __shared__ T hx[TY][4][PP];
    // the halo elements' contributions at their east face (j + P k)
    __shared__ T ch[TY][PP][5];
    // per lattice column of the block: the top level's partial sum (FP64)
    __shared__ double cz[WX * (WY + 1)][5];
    static_assert(NE * NP * 5 <= NE * 7 * NP, "contributions fit the tile");

    const int g = (int)xcd_remap(blockIdx.x, gridDim.x);
    const PenItem &it = B.it[pen_item(B, g, false)];
    const int lb = g - it.boff;
    const uint32_t tq = fdiv((uint32_t)lb, it.fbx);
    const int bx = lb - (int)(tq * it.fbx.d);
    const uint32_t bz = fdiv(tq, it.fby);
    const int by = (int)(tq - bz * it.fby.d);
    const T *D = (const T *)B.D;
    const int layer = it.ni * it.nj;
    const int wz = it.tz * N;
    const bool mainl = (int)threadIdx.x < ML;
    const int exh = (bx == 0 ? it.nx : bx * TX) - 1;  // the element column west of the block

    // Issue the loads of layer ez: main lanes the N+1 nodes of their column,
    // halo lanes their halo nodes (node r: n = h + r HL), every lane the
    // column factors of the metric it needs (main lanes: their column; halo
    // lanes: the halo element's east-face column).  The same loads on every
    // lane, from a dummy address where a lane has nothing to load: no branch,
    // so the compiler's waits on the in-order memory counter stay exact.
    auto gather = [&](int ez, double (*G)[kGather], double *cf) {
        int tid = (int)threadIdx.x;
        asm volatile("" : "+v"(tid));
        int32_t I[P];
        const double *cp;
        if (tid < ML) {
            const int q = tid / PP, c = tid % PP, i = c % P, j = c / P;
            const int ex = bx * TX + q % TX, ey = by * TY + q / TX;
            int gi = ex * N + i, gj = ey * N + j;
            if (gi == it.ni) gi = 0;
            if (gj == it.nj) gj = 0;
            const int base = gi + it.ni * gj + layer * (ez * N);
#pragma unroll
            for (int k = 0; k < P; ++k) I[k] = base + layer * k;
            cp = it.hcol + (int64_t)(ex + it.nx * ey) * (4 * PP) + c;
        } else {
            const int h = tid - ML;
#pragma unroll
            for (int r = 0; r < P; ++r) {
                const int n = h + r * HL;
                I[r] = 0;
                if (r < (HN + HL - 1) / HL && n < HN) {
                    const int y = n / (N * PP), rr = n % (N * PP), m = rr % N, jk = rr / N, jj = jk % P, kk = jk / P;
                    int gj = (by * TY + y) * N + jj;
                    if (gj == it.nj) gj = 0;
                    I[r] = exh * N + m + it.ni * gj + layer * (ez * N + kk);
                }
            }
            const int hy = h < TY * PP ? h / PP : 0, hj = h < TY * PP ? (h % PP) % P : 0;
            cp = it.hcol + (int64_t)(exh + it.nx * (by * TY + hy)) * (4 * PP) + (N + P * hj);
        }
#pragma unroll
        for (int k = 0; k < P; ++k) {
#pragma unroll
            for (int v = 0; v < 5; ++v) G[k][v] = it.qs[I[k] + v * it.nu];
            G[k][5] = it.ref[I[k]];
            G[k][6] = it.ref[I[k] + 2 * it.nu];
        }
#pragma unroll
        for (int f = 0; f < 4; ++f) cf[f] = cp[f * PP];
    };

    double G[P][kGather], cf[4];
    gather((int)bz * it.tz, G, cf);

    for (int L = 0; L < it.tz; ++L) {
        const int ez = (int)bz * it.tz + L;
        // the lane's roles, derived afresh every layer (an opaque copy of the
        // lane index keeps them out of the state carried across layers)
        int tid = (int)threadIdx.x;
        asm volatile("" : "+v"(tid));
        // main lanes: element q = qx + TX qy of the block, column (i, j)
        const int q = tid / PP, c = tid % PP, qx = q % TX, qy = q / TX, i = c % P, j = c / P;
        const int ex = bx * TX + qx, ey = by * TY + qy;
        // halo lanes: h < TY (N+1)^2 computes the halo face node (hj, hk) of block row hy
        const int h = tid - ML;
        const bool hrl = !mainl && h < TY * PP;
        const int hy = hrl ? h / PP : 0, hf = hrl ? h % PP : 0, hj = hf % P, hk = hf / P;
        // summing lanes: lattice column (sa, sb) of the block
        const bool suml = tid < WX * (WY + 1);
        const int sa = tid % WX, sb = tid / WX;
        const int gi = bx * WX + sa, gj = by * WY + sb;
        const bool yseam = sb == 0 || sb == WY;
        const double c0 = cf[0], c1 = cf[1], c2 = cf[2], c3 = cf[3];
        // ---- A1: equation of state, tiles
        // values that live across the barriers are set on every lane and every
        // layer: left unset on the other lanes, the compiler would carry the
        // previous layer's values around the loop in registers
        T irho[P], buoy[P], dz[8][P];
#pragma unroll
        for (int k = 0; k < P; ++k) {
            irho[k] = 0;
            buoy[k] = 0;
#pragma unroll
            for (int f = 0; f < 8; ++f) dz[f][k] = 0;
        }
        if (mainl) {
            T col[8][P];
#pragma unroll
            for (int k = 0; k < P; ++k) {
                const double rp = G[k][0], u = G[k][1], v = G[k][2], w = G[k][3], tp = G[k][4];
                const double rb = G[k][5], tb = it.theta0, pb = G[k][6];
                const double rho = rb + rp;
                const double dl = rp * tb + rb * tp + rp * tp;
                const double pp = pb * eos_rel(dl / (rb * tb), B.gamma, B.eos);
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
                const int l = c + PP * k;
                s[q][0][l] = col[0][k];
                s[q][1][l] = col[1][k];
#pragma unroll
                for (int f = 3; f < 8; ++f) s[q][f - 1][l] = col[f][k];
                if (qx == 0 && i == 0) {
                    const int hl = N + P * j + PP * k;
                    ht[qy][0][hl] = col[0][k];
#pragma unroll
                    for (int f = 3; f < 8; ++f) ht[qy][f - 2][hl] = col[f][k];
                    hx[qy][0][j + P * k] = col[2][k];
                    hx[qy][1][j + P * k] = col[1][k];
                    hx[qy][2][j + P * k] = irho[k];
                    hx[qy][3][j + P * k] = buoy[k];
                }
            }
#pragma unroll
            for (int f = 0; f < 8; ++f)
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    T d = 0;
#pragma unroll
                    for (int m = 0; m < P; ++m) d += D[k * P + m] * col[f][m];
                    dz[f][k] = d;
                }
        } else {
            // the halo elements' nodes with m < N (their face m = N is the block's)
#pragma unroll
            for (int r = 0; r < (HN + HL - 1) / HL; ++r) {
                const int n = h + r * HL;
                if (n < HN) {
                    const int y = n / (N * PP), rr = n % (N * PP), m = rr % N, jk = rr / N, jj = jk % P, kk = jk / P;
                    const double rp = G[r][0], u = G[r][1], v = G[r][2], w = G[r][3], tp = G[r][4];
                    const double rb = G[r][5], tb = it.theta0, pb = G[r][6];
                    const double rho = rb + rp;
                    const double dl = rp * tb + rb * tp + rp * tp;
                    const double pp = pb * eos_rel(dl / (rb * tb), B.gamma, B.eos);
                    const int hl = m + P * jj + PP * kk;
                    ht[y][0][hl] = (T)(rho * u);
                    ht[y][1][hl] = (T)u;
                    ht[y][2][hl] = (T)v;
                    ht[y][3][hl] = (T)w;
                    ht[y][4][hl] = (T)tp;
                    ht[y][5][hl] = (T)pp;
                }
            }
        }
        __syncthreads();  // tiles complete
        // ---- A2: derivatives and R; the summing lanes then issue the loads
        // of the stage update of the nodes they finish in this layer
        T res[P][5];
#pragma unroll
        for (int k = 0; k < P; ++k)
#pragma unroll
            for (int v = 0; v < 5; ++v) res[k][v] = 0;
        if (mainl) {
            T Di[P], Dj[P];
#pragma unroll
            for (int m = 0; m < P; ++m) {
                Di[m] = D[i * P + m];
                Dj[m] = D[j * P + m];
            }
#pragma unroll
            for (int k = 0; k < P; ++k) {
                T mx[10];
                box_node_metric<T>(it.bm, ez, B.xi[k], c0 * B.w[k], c1, c2, c3, mx);
                const int l = c + PP * k;
                const T uu = s[q][2][l], vv = s[q][3][l], ww = s[q][4][l];
                const T Uc0 = uu * mx[0], Uc1 = vv * mx[4], Uc2 = uu * mx[6] + vv * mx[7] + ww * mx[8];
                // the fields one at a time (tile slot sf: 0 rho u, 1 rho v, 2 u, 3 v,
                // 4 w, 5 theta', 6 p'; rho w only along zeta), each adding its
                // terms to R: few values live at once
                T R[5];
#pragma unroll
                for (int f = 0; f < 8; ++f) {
                    T da = 0, db = 0;
                    const T dc = dz[f][k];
                    if (f != 2) {
                        const int sf = f < 2 ? f : f - 1;
#pragma unroll
                        for (int m = 0; m < P; ++m) {
                            if (f != 1) da += Di[m] * s[q][sf][m + P * (j + P * k)];
                            if (f != 0) db += Dj[m] * s[q][sf][i + P * (m + P * k)];
                        }
                    }
                    if (f == 0) R[0] = da * mx[0] + dc * mx[6];                 // d(rho u)/dx
                    if (f == 1) R[0] = R[0] + (db * mx[4] + dc * mx[7]);         // + d(rho v)/dy
                    if (f == 2) R[0] = -(R[0] + dc * mx[8]);                     // + d(rho w)/dz
                    if (f >= 3 && f <= 6) R[f - 2] = -(Uc0 * da + Uc1 * db + Uc2 * dc);
                    if (f == 7) {
                        R[1] = R[1] - (da * mx[0] + dc * mx[6]) * irho[k];
                        R[2] = R[2] - (db * mx[4] + dc * mx[7]) * irho[k];
                        R[3] = R[3] - (dc * mx[8]) * irho[k] + (F64 ? buoy[k] * irho[k] : buoy[k]) * (T)(-B.g0);
                    }
                }
                const bool wall = (ez == 0 && k == 0) || (ez == it.nz - 1 && k == N);
                if (F64 && B.fold && !wall) {
                    const T qv[5] = {buoy[k], uu, vv, ww, s[q][5][l]};
#pragma unroll
                    for (int v = 0; v < 5; ++v) res[k][v] = mx[9] * fma((T)it.cdt, R[v], qv[v]);
                } else {
#pragma unroll
                    for (int v = 0; v < 5; ++v) res[k][v] = mx[9] * R[v];
                }
            }
        }
        __syncthreads();  // tiles read
        // ---- A3: the contributions into LDS, [element][k][column][5]; the halo face
        T *C = &s[0][0][0];
        if (mainl) {
#pragma unroll
            for (int k = 0; k < P; ++k)
#pragma unroll
                for (int v = 0; v < 5; ++v) C[((q * P + k) * PP + c) * 5 + v] = res[k][v];
        }
        if (hrl) {
            // the halo element's contribution at its east-face node (N, hj, hk):
            // xi derivatives from the halo tile, eta and zeta derivatives along
            // the face, which is the block element (0, hy)'s i = 0 face; the
            // face's fields are in ht (m = N) and hx, so this runs while the
            // main lanes overwrite the element tile with their contributions.
            // The fields are walked one at a time, each adding its terms to R
            // (few registers: the main lanes' budget is the kernel's).
            auto face = [&](int f, int jj, int kk) -> T {
                if (f == 1) return hx[hy][1][jj + P * kk];
                if (f == 2) return hx[hy][0][jj + P * kk];
                return ht[hy][f == 0 ? 0 : f - 2][N + P * jj + PP * kk];
            };
            T mx[10];
            box_node_metric<T>(it.bm, ez, B.xi[hk], c0 * B.w[hk], c1, c2, c3, mx);
            const T uu = face(3, hj, hk), vv = face(4, hj, hk), ww = face(5, hj, hk);
            const T ir = hx[hy][2][hf], bu = hx[hy][3][hf];
            const T Uc0 = uu * mx[0], Uc1 = vv * mx[4], Uc2 = uu * mx[6] + vv * mx[7] + ww * mx[8];
            T R[5];
#pragma unroll
            for (int f = 0; f < 8; ++f) {
                T da = 0, db = 0, dc = 0;
                if (f != 1 && f != 2) {
                    const int hf6 = f == 0 ? 0 : f - 2;
#pragma unroll
                    for (int m = 0; m < P; ++m) da += D[N * P + m] * ht[hy][hf6][m + P * hj + PP * hk];
                }
                if (f != 0 && f != 2) {
#pragma unroll
                    for (int m = 0; m < P; ++m) db += D[hj * P + m] * face(f, m, hk);
                }
#pragma unroll
                for (int m = 0; m < P; ++m) dc += D[hk * P + m] * face(f, hj, m);
                if (f == 0) R[0] = da * mx[0] + dc * mx[6];                 // d(rho u)/dx
                if (f == 1) R[0] = R[0] + (db * mx[4] + dc * mx[7]);         // + d(rho v)/dy
                if (f == 2) R[0] = -(R[0] + dc * mx[8]);                     // + d(rho w)/dz
                if (f >= 3 && f <= 6) R[f - 2] = -(Uc0 * da + Uc1 * db + Uc2 * dc);
                if (f == 7) {
                    R[1] = R[1] - (da * mx[0] + dc * mx[6]) * ir;
                    R[2] = R[2] - (db * mx[4] + dc * mx[7]) * ir;
                    R[3] = R[3] - (dc * mx[8]) * ir + (F64 ? bu * ir : bu) * (T)(-B.g0);
                }
            }
            const bool wall = (ez == 0 && hk == 0) || (ez == it.nz - 1 && hk == N);
            if (F64 && B.fold && !wall) {
                const T qv[5] = {bu, uu, vv, ww, face(6, hj, hk)};
#pragma unroll
                for (int v = 0; v < 5; ++v) ch[hy][hf][v] = mx[9] * fma((T)it.cdt, R[v], qv[v]);
            } else {
#pragma unroll
                for (int v = 0; v < 5; ++v) ch[hy][hf][v] = mx[9] * R[v];
            }
        }
        __syncthreads();
        // ---- B: the loads of this layer's stage update and of the next
        // layer's gather go out first (in that order: the memory counter is
        // in order, so waiting for the first does not wait for the second);
        // then every summing lane adds the copies of the nodes of its lattice
        // column (sa, sb) and finishes them
        double fm[P], fn[P][5], fs[P][5], nb[3], nt[3];
        {
            // the operands of the stage update of the nodes finished here:
            // M^-1, q_ref, q_s (walls, or no fold) and the wall normals, from
            // a dummy address (index 0) where a lane does not need them
#pragma unroll
            for (int kk = 0; kk < P; ++kk) {
                const int cl = L * N + kk, gk = ez * N + kk;
                const bool carry = kk == N && L < it.tz - 1;
                const bool zseam = (cl == 0 && (int)bz > 0) || (cl == wz && (int)bz < it.nbz - 1);
                const bool fin = suml && !yseam && !carry && !zseam;
                const bool wall = gk == 0 || gk == it.nk - 1;
                const int32_t I = fin ? gi + it.ni * (gj + it.nj * gk) : 0;
                const int32_t In = fin && B.ca != 0.0 ? I : 0;
                const int32_t Is = fin && B.cb != 0.0 && (wall || !B.fold) ? I : 0;
                fm[kk] = it.Minv[I];
#pragma unroll
                for (int v = 0; v < 5; ++v) {
                    fn[kk][v] = it.qn[In + v * it.nu];
                    fs[kk][v] = it.qs[Is + v * it.nu];
                }
            }
            const int hb = suml && !yseam ? gi + it.ni * gj : 0;  // horizontal index of the column
            const double *pb = it.nrm + ((ez == 0) ? hb : 0);
            const double *pt = it.nrm + 3 * it.nh + ((ez == it.nz - 1) ? hb : 0);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                nb[d] = pb[d * it.nh];
                nt[d] = pt[d * it.nh];
            }
        }
        // the next layer (the last layer loads its own layer again: G stays
        // defined on every path, so it is not carried through the layer)
        gather(L + 1 < it.tz ? ez + 1 : ez, G, cf);
        if (suml) {
            // x copies: (element column qx, local i); halo = the western neighbour
            int xq[2], xi_[2], nxc;
            bool xh = false;
            if (sa == 0) {
                xq[0] = 0; xi_[0] = 0; xh = true; nxc = 2;
                xq[1] = 0; xi_[1] = N;
            } else if (sa % N == 0) {
                xq[0] = sa / N; xi_[0] = 0; xq[1] = sa / N - 1; xi_[1] = N; nxc = 2;
            } else {
                xq[0] = sa / N; xi_[0] = sa % N; xq[1] = xq[0]; xi_[1] = xi_[0]; nxc = 1;
            }
            int yq[2], yj[2], nyc;
            if (sb == 0) {
                yq[0] = 0; yj[0] = 0; nyc = 1;
            } else if (sb == WY) {
                yq[0] = TY - 1; yj[0] = N; nyc = 1;
            } else if (sb % N == 0) {
                yq[0] = sb / N; yj[0] = 0; yq[1] = sb / N - 1; yj[1] = N; nyc = 2;
            } else {
                yq[0] = sb / N; yj[0] = sb % N; nyc = 1;
            }
            if (nyc == 1) { yq[1] = yq[0]; yj[1] = yj[0]; }
#pragma unroll
            for (int kk = 0; kk < P; ++kk) {
                double r[5] = {0, 0, 0, 0, 0};
                if (kk == 0 && L > 0) {
#pragma unroll
                    for (int v = 0; v < 5; ++v) r[v] = cz[tid][v];
                }
                for (int y = 0; y < nyc; ++y)
                    for (int x = 0; x < nxc; ++x) {
                        const T *src = (x == 1 && xh) ? &ch[yq[y]][yj[y] + P * kk][0]
                                                      : C + (((yq[y] * TX + xq[x]) * P + kk) * PP + xi_[x] + P * yj[y]) * 5;
#pragma unroll
                        for (int v = 0; v < 5; ++v) r[v] += (double)src[v];
                    }
                if (kk == N && L < it.tz - 1) {
                    // the top level is the next layer's bottom level: carry its sum
#pragma unroll
                    for (int v = 0; v < 5; ++v) cz[tid][v] = r[v];
                    continue;
                }
                const int cl = L * N + kk;  // level in the block, 0..wz
                const int gk = ez * N + kk;
                const bool zseam = (cl == 0 && (int)bz > 0) || (cl == wz && (int)bz < it.nbz - 1);
                if (yseam) {
                    double *dst = it.py + ((((int64_t)(by * 2 + (sb == WY)) * it.nbz + bz) * (wz + 1) + cl) * it.ni + gi) * 5;
#pragma unroll
                    for (int v = 0; v < 5; ++v) dst[v] = r[v];
                } else if (zseam) {
                    double *dst = it.pz + ((((int64_t)bz * 2 + (cl == wz)) * it.nj + gj) * it.ni + gi) * 5;
#pragma unroll
                    for (int v = 0; v < 5; ++v) dst[v] = r[v];
                } else {
                    // M^-1, wall projection and stage update (as pen_finish)
                    const int32_t I = gi + it.ni * (gj + it.nj * gk);
                    const bool wall = gk == 0 || gk == it.nk - 1;
                    const StageCoef sc{B.ca, B.cb, it.cdt};
#pragma unroll
                    for (int v = 0; v < 5; ++v) r[v] *= fm[kk];
                    double o[5];
                    if (B.fold && !wall) {
#pragma unroll
                        for (int v = 0; v < 5; ++v) it.qout[I + v * it.nu] = o[v] = rk_update_folded(sc, fn[kk][v], r[v]);
                    } else {
                        if (wall) {
                            const double n0 = gk == 0 ? nb[0] : nt[0], n1 = gk == 0 ? nb[1] : nt[1],
                                         n2 = gk == 0 ? nb[2] : nt[2];
                            const double dn = r[1] * n0 + r[2] * n1 + r[3] * n2;
                            r[1] -= dn * n0;
                            r[2] -= dn * n1;
                            r[3] -= dn * n2;
                        }
#pragma unroll
                        for (int v = 0; v < 5; ++v) it.qout[I + v * it.nu] = o[v] = rk_update(sc, fn[kk][v], fs[kk][v], r[v]);
                    }
                    flag_nonfinite(it.flag, o, 5);
                }
            }
        }
        __syncthreads();  // contributions read before the next layer's tiles
    }
}

// Finish of the nodes on the blocks' y faces (every level) and z faces (the
// other rows): the sum of their blocks' partial sums, in a fixed order.  A
// row of lanes runs along x, so state reads and writes are contiguous.
template <int N>
__global__ __launch_bounds__(kSeamThreads) void k_pencil_seam(PenBatch B)
{
    constexpr int WY = pen_ty<N>() * N;
    const int g = (int)xcd_remap(blockIdx.x, gridDim.x);
    const PenItem &it = B.it[pen_item(B, g, true)];
    const int lb = g - it.soff;
    const int row = lb / it.sblk;
    const int gi = (lb - row * it.sblk) * kSeamThreads + (int)threadIdx.x;
    if (gi >= it.ni) return;
    const int wz = it.tz * N;
    double r[5] = {0, 0, 0, 0, 0};
    int gj, gk;
    auto add = [&](const double *src) {
#pragma unroll
        for (int v = 0; v < 5; ++v) r[v] += src[v];
    };
    auto pyp = [&](int by, int f, int bz, int cl) {
        return it.py + ((((int64_t)(by * 2 + f) * it.nbz + bz) * (wz + 1) + cl) * it.ni + gi) * 5;
    };
    if (row < it.nby * it.nk) {  // y face: the north face of block row by - 1 and the south face of by
        gk = row / it.nby;
        const int by = row - gk * it.nby, bs = by == 0 ? it.nby - 1 : by - 1;
        gj = by * WY;
        if (gk % wz == 0 && gk > 0 && gk < it.nk - 1) {  // also a z face: four blocks
            const int bz = gk / wz;
            add(pyp(by, 0, bz, 0));
            add(pyp(bs, 1, bz, 0));
            add(pyp(by, 0, bz - 1, wz));
            add(pyp(bs, 1, bz - 1, wz));
        } else {
            int bz = gk / wz;
            if (bz >= it.nbz) bz = it.nbz - 1;
            const int cl = gk - bz * wz;
            add(pyp(by, 0, bz, cl));
            add(pyp(bs, 1, bz, cl));
        }
    } else {  // z face between block layers bz - 1 and bz, rows off the y faces
        const int r2 = row - it.nby * it.nk, nr = it.nj - it.nby;
        const int bz = 1 + r2 / nr, jr = r2 - (bz - 1) * nr;
        gj = (jr / (WY - 1)) * WY + 1 + jr % (WY - 1);
        gk = bz * wz;
        add(it.pz + ((((int64_t)bz * 2 + 0) * it.nj + gj) * it.ni + gi) * 5);
        add(it.pz + ((((int64_t)(bz - 1) * 2 + 1) * it.nj + gj) * it.ni + gi) * 5);
    }
    const int32_t I = gi + it.ni * (gj + it.nj * gk);
    pen_finish(it, B, I, r, gk == 0 || gk == it.nk - 1);
}

// element layers per block: the tallest block (a divisor of nz) that still
// gives the mesh at least kTargetBlocks blocks, so that one mesh alone fills
// the GPU; a function of the mesh only, so a mesh's rounding does not depend
// on its batch
constexpr int kTargetBlocks = 512;

template <int N>
int pen_tz(const Mesh &m)
{
    const int64_t cols = (int64_t)(m.d.ne[0] / pen_tx<N>()) * (m.d.ne[1] / pen_ty<N>());
    const int nz = m.d.ne[2];
    for (int tz = nz; tz >= 1; --tz)
        if (nz % tz == 0 && cols * (nz / tz) >= kTargetBlocks) return tz;
    return 1;
}

template <int N>
uint64_t pen_partial_bytes(const Mesh &m, int tz)
{
    const int64_t nby = m.d.ne[1] / pen_ty<N>(), nbz = m.d.ne[2] / tz, wz = (int64_t)tz * N;
    const uint64_t py = 40ull * nby * 2 * nbz * (wz + 1) * m.ni;
    const uint64_t pz = nbz > 1 ? 40ull * nbz * 2 * m.nj * m.ni : 0;
    return ((py + 255) & ~uint64_t(255)) + pz;
}

template <int N>
bool pen_mesh_ok(const Mesh &m, int32_t prec)
{
    if (m.stage_mode != NUMA_STAGE_BLOCK) return false;
    if (m.d.kind != NUMA_MESH_BOX || !m.walls || m.metric_mode != NUMA_METRIC_RECOMPUTE) return false;
    if (m.d.ne[0] % pen_tx<N>() || m.d.ne[1] % pen_ty<N>()) return false;
    const uint64_t ev = (prec == NUMA_PREC_MIXED ? 20ull : 40ull) * m.nl;
    return pen_partial_bytes<N>(m, pen_tz<N>(m)) <= ev;
}

template <int N, typename T>
int32_t pen_chunk(const StepItem *items, int n, int phase, hipStream_t s)
{
    PenBatch B;
    B.n = n;
    B.ca = items[0].c.a;
    B.cb = items[0].c.b;
    B.fold = (std::is_same<T, double>::value && B.cb != 0.0) ? 1 : 0;
    B.gamma = items[0].mesh->gamma;
    B.g0 = items[0].mesh->ph.g0;
    B.D = std::is_same<T, float>::value ? (const void *)items[0].mesh->dv.D32 : (const void *)items[0].mesh->dv.D64;
    B.xi = items[0].mesh->dv.xi64;
    B.w = items[0].mesh->dv.w64;
    eos_coeffs(B.gamma, B.eos);
    int64_t bo = 0, so = 0;
    for (int k = 0; k < n; ++k) {
        const Mesh &m = *items[k].mesh;
        PenItem &it = B.it[k];
        const int tz = pen_tz<N>(m);
        it.qs = items[k].qs;
        it.qout = items[k].qout;
        it.qn = items[k].qn;
        it.ref = m.dv.ref;
        it.Minv = stage_minv(m);
        it.nrm = m.dv.nrm;
        it.hcol = m.dv.hcol;
        it.py = (double *)items[k].ev;
        it.flag = items[k].flag;
        it.nu = m.nu;
        it.nh = m.nh;
        it.ni = (int)m.ni;
        it.nj = (int)m.nj;
        it.nk = (int)m.nk;
        it.nx = m.d.ne[0];
        it.ny = m.d.ne[1];
        it.nz = m.d.ne[2];
        it.nbx = it.nx / pen_tx<N>();
        it.nby = it.ny / pen_ty<N>();
        it.tz = tz;
        it.nbz = it.nz / tz;
        const int64_t wz = (int64_t)tz * N;
        const uint64_t pyb = 40ull * it.nby * 2 * it.nbz * (wz + 1) * it.ni;
        it.pz = (double *)((char *)items[k].ev + ((pyb + 255) & ~uint64_t(255)));
        it.fbx = fast_div((uint32_t)it.nbx);
        it.fby = fast_div((uint32_t)it.nby);
        it.cdt = items[k].c.cdt;
        it.theta0 = m.ph.T0;
        it.bm = box_metric(m);
        it.boff = (int)bo;
        it.soff = (int)so;
        it.srows = it.nby * it.nk + (it.nbz - 1) * (it.nj - it.nby);
        it.sblk = (it.ni + kSeamThreads - 1) / kSeamThreads;
        bo += (int64_t)it.nbx * it.nby * it.nbz;
        so += (int64_t)it.srows * it.sblk;
    }
    if (bo >= (int64_t(1) << 31) || so >= (int64_t(1) << 31)) {
        set_error("batch: more than 2^31 - 1 workgroups in one launch");
        return NUMA_EUNSUPPORTED;
    }
    for (int k = n; k < kMaxPenBatch; ++k) B.it[k] = PenItem{};
    if (phase == 0)
        hipLaunchKernelGGL((k_pencil<N, T>), dim3((unsigned)bo), dim3(pen_threads<N>()), 0, s, B);
    else
        hipLaunchKernelGGL((k_pencil_seam<N>), dim3((unsigned)so), dim3(kSeamThreads), 0, s, B);
    NUMA_HIP(hipGetLastError());
    return NUMA_OK;
}

template <typename T>
int32_t pen_stage_t(const StepItem *items, int n, int phase, hipStream_t s)
{
    for (int c0 = 0; c0 < n; c0 += kMaxPenBatch) {
        const int c = n - c0 < kMaxPenBatch ? n - c0 : kMaxPenBatch;
        int32_t rc;
        switch (items[0].mesh->N) {
        case 2: rc = pen_chunk<2, T>(items + c0, c, phase, s); break;
        case 3: rc = pen_chunk<3, T>(items + c0, c, phase, s); break;
        default: rc = pen_chunk<4, T>(items + c0, c, phase, s); break;
        }
        if (rc) return rc;
    }
    return NUMA_OK;
}

}  // namespace

bool pencil_ok(const Mesh &m, int32_t prec)
{
    switch (m.N) {
    case 2: return pen_mesh_ok<2>(m, prec);
    case 3: return pen_mesh_ok<3>(m, prec);
    case 4: return pen_mesh_ok<4>(m, prec);
    default: return false;
    }
}

int32_t launch_pencil_stage(const StepItem *items, int n, int32_t prec, int phase, hipStream_t s)
{
    if (prec == NUMA_PREC_MIXED) return pen_stage_t<float>(items, n, phase, s);
    return pen_stage_t<double>(items, n, phase, s);
}

}  // namespace numa
