// Batched fused stages on box meshes: the elements and nodes of several
// independent solves of the same order advance together, one element launch
// and one finish launch per stage for the whole batch (continuous batching of
// ensemble members and regional solves).  Each item brings its own state and
// private scratch; geometry may be shared between items.  The per-element
// and per-node arithmetic is the single-mesh code (kernels.h), so an item's
// result does not depend on what it is batched with.  A single box mesh
// (numa_step) runs through the same kernels with one item.
#include <type_traits>

#include "kernels.h"

namespace numa {
namespace {

using namespace dev;

constexpr int kMaxBatch = 16;  // items per launch (kernel-argument table)

struct BatchItem {
    const double *qs;  // stage input state [5][nu]
    double *qout;      // stage output state
    const double *qn;  // state at the start of the step
    const double *ref, *Minv, *nrm;
    const void *met;      // [ne][10][np] of T
    void *ev;             // [nl][5] of T: contributions of this stage, node-major
    const double *hcol;   // column factors of the recomputed metric
    int64_t nu, nh;
    int ni, nj, nkw;      // lattice extents; nkw: extent in z when periodic, else -1
    int nz, walls;
    int mblk;             // finish blocks of the main layers: (nx/SEG) ny nz
    FastDiv fx, fy, fseg;  // division by nx, ny and nx/SEG
    double dt;
    BoxMetric bm;          // constants of the recomputed metric
    int eoff, boff;        // first element / finish block of this item in the launch
};

struct Batch {
    int n, stage;
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

template <int N, typename T, int GEO>
__global__ __launch_bounds__(block_threads<N>()) void k_elem_batch(Batch B)
{
    constexpr int NP = (N + 1) * (N + 1) * (N + 1), BT = block_threads<N>();
    __shared__ T s[8][NP];
    const int g = (int)xcd_remap(blockIdx.x, gridDim.x);
    const BatchItem &it = B.it[batch_item(B, g, false)];
    const int e = g - it.eoff;
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
    a.bm = it.bm;
#pragma unroll
    for (int c = 0; c < kEosTerms; ++c) a.eos[c] = B.eos[c];
    a.xi = B.xi;
    a.w = B.w;
    a.Dd = B.Dd;
    NodeOut<T> o;
    const int l = threadIdx.x;
    const bool act = element_rhs<N, T, false, GEO>(a, e, l, s, o);
    // node-major [n_local][5] output (a copy's five values in one run for the
    // finish), staged through the tile so that the block writes its 5 (N+1)^3
    // values as one contiguous, coalesced run
    __syncthreads();  // every lane has finished reading the tile
    T *st = &s[0][0];
    if (act) {
#pragma unroll
        for (int v = 0; v < 5; ++v) st[l * 5 + v] = o.Jw * o.R[v];
    }
    __syncthreads();
    T *out = (T *)it.ev + (int64_t)e * (NP * 5);
#pragma unroll
    for (int r = 0; r < (NP * 5 + BT - 1) / BT; ++r) {
        const int t = l + r * BT;
        if (t < NP * 5) out[t] = st[t];
    }
}

template <int N, int SEG, typename T>
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
    box_finish_node<N, SEG, T>(p, b, (const T *)it.ev, sx, ey, kbase == 0 ? (int)ez : it.nz - 1, threadIdx.x, kbase,
                               klayers, B.stage, it.dt, it.qn, it.qs, it.qout);
}

template <int N, typename T>
int32_t run_chunk(const StepItem *items, int n, int stage, int phase, hipStream_t s)
{
    constexpr int SEG = seg_for<N>();
    Batch B;
    B.n = n;
    B.stage = stage;
    B.gamma = items[0].mesh->gamma;
    B.g0 = items[0].mesh->ph.g0;
    B.D = std::is_same<T, float>::value ? (const void *)items[0].mesh->dv.D32 : (const void *)items[0].mesh->dv.D64;
    B.xi = items[0].mesh->dv.xi64;
    B.w = items[0].mesh->dv.w64;
    B.Dd = items[0].mesh->dv.D64;
    eos_coeffs(B.gamma, B.eos);
    int64_t eo = 0, bo = 0;
    for (int k = 0; k < n; ++k) {
        const Mesh &m = *items[k].mesh;
        BatchItem &it = B.it[k];
        it.qs = items[k].qs;
        it.qout = items[k].qout;
        it.qn = items[k].qn;
        it.ref = m.dv.ref;
        it.Minv = m.dv.Minv;
        it.nrm = m.dv.nrm;
        it.met = std::is_same<T, float>::value ? (const void *)m.dv.met32 : (const void *)m.dv.met;
        it.ev = items[k].ev;
        it.hcol = m.dv.hcol;
        it.nu = m.nu;
        it.nh = m.nh;
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
        it.dt = items[k].dt;
        it.bm = box_metric(m);
        it.eoff = (int)eo;
        it.boff = (int)bo;
        eo += m.ne;
        bo += mblk + (m.walls ? (int64_t)(m.d.ne[0] / SEG) * m.d.ne[1] : 0);
    }
    if (eo >= (int64_t(1) << 31) || bo >= (int64_t(1) << 31)) {
        set_error("batch: more than 2^31 - 1 elements in one launch");
        return NUMA_EUNSUPPORTED;
    }
    for (int k = n; k < kMaxBatch; ++k) B.it[k] = BatchItem{};
    if (phase == 0) {
        if (items[0].mesh->metric_mode == NUMA_METRIC_RECOMPUTE)
            hipLaunchKernelGGL((k_elem_batch<N, T, kMetricBox>), dim3((unsigned)eo), dim3(block_threads<N>()), 0, s, B);
        else
            hipLaunchKernelGGL((k_elem_batch<N, T, kMetricStored>), dim3((unsigned)eo), dim3(block_threads<N>()), 0, s,
                               B);
    } else {
        const int threads = ((SEG * N * N * N + 63) / 64) * 64;
        hipLaunchKernelGGL((k_fin_batch<N, SEG, T>), dim3((unsigned)bo), dim3(threads), 0, s, B);
    }
    NUMA_HIP(hipGetLastError());
    return NUMA_OK;
}

template <typename T>
int32_t run_stage_t(const StepItem *items, int n, int stage, int phase, hipStream_t s)
{
    for (int c0 = 0; c0 < n; c0 += kMaxBatch) {
        const int c = n - c0 < kMaxBatch ? n - c0 : kMaxBatch;
        int32_t rc;
        switch (items[0].mesh->N) {
        case 1: rc = run_chunk<1, T>(items + c0, c, stage, phase, s); break;
        case 2: rc = run_chunk<2, T>(items + c0, c, stage, phase, s); break;
        case 3: rc = run_chunk<3, T>(items + c0, c, stage, phase, s); break;
        case 4: rc = run_chunk<4, T>(items + c0, c, stage, phase, s); break;
        case 5: rc = run_chunk<5, T>(items + c0, c, stage, phase, s); break;
        case 6: rc = run_chunk<6, T>(items + c0, c, stage, phase, s); break;
        case 7: rc = run_chunk<7, T>(items + c0, c, stage, phase, s); break;
        default: rc = run_chunk<8, T>(items + c0, c, stage, phase, s); break;
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

int32_t launch_batch_stage(const StepItem *items, int n, int32_t prec, int32_t stage, int phase, hipStream_t s)
{
    if (prec == NUMA_PREC_MIXED) return run_stage_t<float>(items, n, stage, phase, s);
    return run_stage_t<double>(items, n, stage, phase, s);
}

}  // namespace numa
