// Internal declarations of libnuma: the host mesh, the workspace layout and
// the kernel-launch entry points shared by the HIP translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "numa.h"

namespace numa {

constexpr int kMaxP = 9;  // N <= 8

void set_error(const char *fmt, ...);

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.
// Remap the block index so that every XCD walks one contiguous range of the
// work items (elements or unique nodes): neighbours that share cache lines are
// then fetched once into the same L2 instead of once per XCD.
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nblocks)
{
    const int64_t q = nblocks / kXcds, r = nblocks % kXcds;
    const int64_t x = b % kXcds, slot = b / kXcds;
    return x * q + (x < r ? x : r) + slot;
}

// Division by a run-time invariant divisor d >= 1 with one high multiply
// (Granlund and Montgomery, "Division by invariant integers using
// multiplication", PLDI 1994, Fig. 4.1): with l = ceil(log2 d),
// m = floor(2^32 (2^l - d) / d) + 1, s1 = min(l, 1), s2 = max(l - 1, 0),
// n / d = (t + ((n - t) >> s1)) >> s2 where t = mulhi(m, n), exact for every
// 32-bit n.  The element and finish kernels decompose their block index this
// way instead of with 64-bit divisions.
struct FastDiv {
    uint32_t d, m, s1, s2;
};

inline FastDiv fast_div(uint32_t d)
{
    FastDiv f{};
    uint32_t l = 0;
    while ((uint64_t(1) << l) < d) ++l;
    f.d = d;
    f.m = (uint32_t)(((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1);
    f.s1 = l < 1 ? l : 1;
    f.s2 = l > 1 ? l - 1 : 0;
    return f;
}

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv &f)
{
    const uint32_t t = __umulhi(f.m, n);
    return (t + ((n - t) >> f.s1)) >> f.s2;
}

// Returns NUMA_EDEVICE (with the message recorded) if a HIP call failed.
#define NUMA_HIP(call)                                                                        \
    do {                                                                                      \
        hipError_t _e = (call);                                                               \
        if (_e != hipSuccess) {                                                               \
            ::numa::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(_e), __FILE__, \
                              __LINE__);                                                      \
            return NUMA_EDEVICE;                                                              \
        }                                                                                     \
    } while (0)

// Device pointers into the caller's workspace.
struct DeviceView {
    int32_t *G = nullptr;      // [n_elem][np] gather map
    int32_t *off = nullptr;    // [n_unique+1] inverse map offsets
    int32_t *idx = nullptr;    // [n_local] copies (e*np + l), ascending per unique node
    int32_t *hlat = nullptr;   // shell: [n_horiz][3] surface lattice of each horizontal node
    double *met = nullptr;     // [n_elem][10][np] inverse metric (9) and J w
    float *met32 = nullptr;    // same, FP32 (mixed path)
    double *ref = nullptr;     // [3][n_unique] rho_bar, theta_bar, p_bar
    double *M = nullptr;       // [n_unique]
    double *Minv = nullptr;    // [n_unique]
    double *MinvR = nullptr;   // [n_unique] 1 / (sum of the copies' recomputed J w): the mass of the
                               // recomputed metric's kernels (box: c0 w_k; shell: column x layer factor)
    double *grav = nullptr;    // shell: [3][n_unique]
    double *nrm = nullptr;     // [2][3][n_horiz] bottom and top wall normals
    double *xu = nullptr;      // [3][n_unique] unique coordinates
    double *hcol = nullptr;    // box: [nx*ny][4][(N+1)^2] column factors of the recomputed metric
    double *scol = nullptr;    // shell: [6 ne^2][13][(N+1)^2] column factors of the recomputed metric
    double *slay = nullptr;    // shell: [nz (N+1)][4] layer factors of the recomputed metric
    int32_t *shid = nullptr;   // shell: [6 ne^2][(N+1)^2] horizontal unique id of each element column
    int32_t *hoff = nullptr;   // shell: [n_horiz+1] offsets of the horizontal copy lists
    int32_t *hidx = nullptr;   // shell: [6 ne^2 (N+1)^2] copies e*np + l (bottom layer, k = 0), ascending
    int32_t *own = nullptr;    // [n_unique] unique ids in first-occurrence order of the element scan
    int32_t *toff = nullptr;   // [n_unique+1] copy offsets in that order
    int32_t *tidx = nullptr;   // [n_local] copies (e*np + l), ascending per node, in that order
    double *ev64 = nullptr;    // [5][n_local] element contributions of a fused stage, FP64 path
    float *ev32 = nullptr;     // same, mixed path
    double *qs = nullptr;      // [5][n_unique] stage state scratch
    double *qs2 = nullptr;     // [5][n_unique] second stage state (SSP-RK(5,3) keeps u_2; IMEX line vectors)
    double *imexLU = nullptr;  // box, workspace bit 2: [n_levels][4N+1][n_horiz] IMEX line factors
    double *D64 = nullptr;     // [(N+1)^2] derivative matrix
    double *xi64 = nullptr;    // [N+1] GLL nodes
    double *w64 = nullptr;     // [N+1] GLL weights
    float *D32 = nullptr;      // same, FP32
    int32_t *flag = nullptr;   // one int: the geometry's non-positive-Jacobian flag
};

struct Mesh {
    numa_mesh_desc d{};
    int N = 0, P = 0, np = 0;
    int64_t ne = 0, nl = 0, nu = 0, nh = 0, nk = 0;
    int64_t ni = 0, nj = 0;  // box lattice extents
    bool walls = false;      // no-flux bottom and top
    double xi[kMaxP]{}, w[kMaxP]{}, D[kMaxP * kMaxP]{};
    std::vector<int32_t> G, off, idx, hlat;
    std::vector<float> D32;
    std::vector<int32_t> own, toff, tidx;
    std::vector<int32_t> hoff, hidx;  // shell: copies of each horizontal node in the bottom layer (e*np + l)
    // optional event timing of the stage kernels (numa_profile)
    bool profiling = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, int>> ev_elem, ev_fin;  // indices into ev_pool
    size_t ev_used = 0;
    // workspace
    char *ws = nullptr;
    uint64_t ws_bytes = 0;
    int32_t prec_mask = 0;
    bool lean = false;  // NUMA_WS_LEAN: only what batched recomputed-metric steps read
    DeviceView dv;
    bool uploaded = false, geom = false;
    int metric_mode = 0;  // NUMA_METRIC_STORED or NUMA_METRIC_RECOMPUTE (box)
    int stage_mode = NUMA_STAGE_AUTO;  // NUMA_STAGE_* (box)
    int integrator = 0;         // NUMA_RK_SSP33 or NUMA_RK_SSP53
    double imex_dt = 0.0;       // dt of the IMEX factors in the workspace (valid when imex_ok)
    bool imex_ok = false;
    bool filter_on = false;     // numa_step applies the filter after every step
    double filter_order = 0.0;  // Boyd-Vandeven order p
    int filter_cutoff = 0;      // modes 0..cutoff pass unchanged
    numa_phys ph{};
    double gamma = 0.0;
    // numa_step's captured step: the launches of one step (stages, filter)
    // recorded once on cap_stream and replayed per step; valid while the
    // precision, dt, state and settings generation match
    bool step_graphs = true;
    uint64_t gen = 0;  // bumped by every call that changes what a step launches
    hipStream_t cap_stream = nullptr;
    hipGraph_t step_graph = nullptr;
    hipGraphExec_t step_exec = nullptr;
    int32_t g_prec = -1;
    double g_dt = 0.0;
    const double *g_q = nullptr;
    uint64_t g_gen = 0;
};

// Host GLL (nodes, weights, derivative matrix); returns false for bad order.
bool gll(int N, double *xi, double *w, double *D);

// Host mesh construction (numbering, gather map, inverse map).
int32_t build_mesh(Mesh &m);

// Workspace layout: computes byte offsets, fills dv when base != nullptr.
uint64_t layout_workspace(Mesh &m, int32_t prec_mask, char *base);

// Kernel launchers (return NUMA_OK or NUMA_EDEVICE).
int32_t launch_geometry(Mesh &m, hipStream_t s);
int32_t launch_export(Mesh &m, int32_t what, void *out, hipStream_t s);
int32_t launch_init_state(Mesh &m, const numa_ic &ic, const double *noise, double *q, hipStream_t s);
int32_t launch_rhs(Mesh &m, int32_t prec, const double *q, double *evec, hipStream_t s);
// minv: the inverse mass applied with NUMA_DSS_MASS (null: the stored metric's M^-1)
int32_t launch_dss(Mesh &m, int32_t nvar, const double *cin, double *out, int32_t flags, hipStream_t s,
                   const double *minv = nullptr);
void filter_sigma(int N, double order, int32_t cutoff, double *sigma);
void filter_matrix(int N, const double *xi, const double *w, double order, int32_t cutoff, double *F);
int32_t launch_filter(Mesh &m, double order, int32_t cutoff, double *q, hipStream_t s);
// the filter of a box whose FP64 stages take the split DSS, through the same
// DSS (column element kernel, face finish); F: the 1D nodal filter matrix
bool filter_split_ok(const Mesh &m);
int32_t launch_filter_split(const Mesh &m, const double *F, double *q, hipStream_t s);
int32_t launch_box_plain_finish(const Mesh &m, const double *ev, double *q, hipStream_t s);
int32_t launch_shell_plain_finish(Mesh &m, const double *ev, double *q, hipStream_t s);
uint64_t imex_lds_bytes(const Mesh &m);
uint64_t imex_factor_bytes(const Mesh &m);
int32_t launch_imex_factor(Mesh &m, double dt, hipStream_t s);
int32_t launch_imex_correction(Mesh &m, double dt, double ra, double *qprev, double *qcur, hipStream_t s);
// The update of one Runge-Kutta stage in Shu-Osher form, written as
// q_out = a q_ref + b (q_s + cdt R): a is the weight of the reference state
// (q^n or an earlier stage; not read when a = 0), b the weight of the stage
// the right-hand side R was taken from, cdt = (beta / b) dt.  b = 0 means
// q_out = a q_ref + cdt R (the explicit leap-frog step).
struct StageCoef {
    double a, b, cdt;
};
StageCoef ssp33_stage(int stage, double dt);

int32_t launch_rk_stage(Mesh &m, int32_t stage, double dt, const double *qn, const double *qs,
                        const double *r, double *qout, hipStream_t s);
// One solve of a batch at one stage: states and the E-vector scratch.
struct StepItem {
    const Mesh *mesh;
    const double *qn, *qs;   // qn: the stage's reference state
    double *qout;
    void *ev;
    StageCoef c;
    int32_t *flag = nullptr;  // device: set to 1 when the stage writes a non-finite value
};

// Box meshes whose x extent fits the finish block's segment take the batched
// kernels; phase 0 launches the element kernels, phase 1 the finish kernels.
bool box_batchable(const Mesh &m);
// the mesh's stages of precision prec run the split DSS (NUMA_STAGE_SPLIT,
// or NUMA_STAGE_AUTO in FP64)
bool split_ok(const Mesh &m, int32_t prec);
// ... through the batched kernels: box_batchable, or the split DSS, which
// takes any box x extent
inline bool stage_batched(const Mesh &m, int32_t prec) { return box_batchable(m) || split_ok(m, prec); }
int32_t launch_batch_stage(const StepItem *items, int n, int32_t prec, int phase, hipStream_t s);

// Batched steps (api.cpp), shared by numa_step_batch and the no-allocation
// variant: argument checks (own_scratch: each item brings its scratch, else
// the library supplies it), the scratch the items need laid out one after
// another, the stages of the items' integrator, and the run itself (pool:
// null for the items' own scratch; st: stages x n stage items).
int32_t check_batch(const numa_batch_item *items, int32_t n, int32_t prec, bool own_scratch, const char *fn);
uint64_t batch_pool_bytes(const numa_batch_item *items, int32_t n, int32_t prec);
int batch_stages(const numa_batch_item *items);
int32_t run_step_batch(const numa_batch_item *items, int32_t n, int32_t prec, int32_t nsteps, char *pool,
                       StepItem *st, hipStream_t s);

// The fused block stage (pencil.hip): box meshes with walls, recomputed
// metric, N = 2..4, nx and ny multiples of the block; phase 0 launches the
// block kernel, phase 1 the kernel of the nodes shared between blocks.  The
// stage's input and output states must be distinct.
bool pencil_ok(const Mesh &m, int32_t prec);
inline bool pencil_stage_ok(const StepItem &it, int32_t prec)
{
    return it.qs != it.qout && pencil_ok(*it.mesh, prec);
}
int32_t launch_pencil_stage(const StepItem *items, int n, int32_t prec, int phase, hipStream_t s);

int32_t launch_stage_elements(Mesh &m, int32_t prec, const StageCoef &c, const double *qs, hipStream_t s);
// the shell's FP64 stages that use q_s (b != 0) fold it into the node-major
// contributions away from the bottom and top layers (k_rhs, k_shell_finish)
inline bool shell_folds(const Mesh &m, int32_t prec, const StageCoef &c)
{
    return m.d.kind == NUMA_MESH_SHELL && prec != NUMA_PREC_MIXED && c.b != 0.0;
}
int32_t launch_stage_finish(Mesh &m, int32_t prec, const StageCoef &c, const double *qn, const double *qs,
                            double *qout, hipStream_t s);

}  // namespace numa
