// C-ABI entry points of libnuma (declared in include/numa.h): argument
// checking, error reporting, workspace binding and the stage sequencing of
// numa_step.  All arithmetic of the path runs in the HIP kernels.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "numa_internal.h"

namespace numa {

static thread_local char g_err[512] = "no error";

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

}  // namespace numa

using numa::Mesh;
using numa::set_error;

struct numa_mesh : Mesh {};
struct numa_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

static inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

static int32_t need_ready(numa_mesh_t m, const char *fn)
{
    if (!m) {
        set_error("%s: null mesh handle", fn);
        return NUMA_EINVAL;
    }
    if (!m->ws) {
        set_error("%s: no workspace attached", fn);
        return NUMA_ENOMEM;
    }
    if (!m->geom) {
        set_error("%s: numa_geometry has not run on this mesh", fn);
        return NUMA_EINVAL;
    }
    return NUMA_OK;
}

// the entry points that read the per-node metric, the gather map or the
// mesh's own scratch: not on a lean workspace
static int32_t need_full(numa_mesh_t m, const char *fn)
{
    if (m->lean) {
        set_error("%s: the workspace was attached lean (NUMA_WS_LEAN): only the batched steps of the recomputed "
                  "metric run on it", fn);
        return NUMA_ENOMEM;
    }
    return NUMA_OK;
}

static int32_t check_prec(numa_mesh_t m, int32_t prec, const char *fn)
{
    if (prec != NUMA_PREC_FP64 && prec != NUMA_PREC_MIXED) {
        set_error("%s: unknown precision %d", fn, prec);
        return NUMA_EINVAL;
    }
    if (prec == NUMA_PREC_MIXED && !(m->prec_mask & 2)) {
        set_error("%s: mixed precision needs a workspace attached with prec_mask bit 1", fn);
        return NUMA_EINVAL;
    }
    return NUMA_OK;
}

extern "C" {

const char *numa_last_error(void) { return numa::g_err; }

int32_t numa_gll(int32_t order, double *xi, double *w, double *D)
{
    if (!xi || !w || !D) {
        set_error("numa_gll: null output");
        return NUMA_EINVAL;
    }
    if (!numa::gll(order, xi, w, D)) {
        set_error("numa_gll: order %d outside 1..8", order);
        return NUMA_EINVAL;
    }
    return NUMA_OK;
}

int32_t numa_mesh_create(const numa_mesh_desc *d, numa_mesh_t *out)
{
    if (!d || !out) {
        set_error("numa_mesh_create: null argument");
        return NUMA_EINVAL;
    }
    *out = nullptr;
    numa_mesh *m = new (std::nothrow) numa_mesh();
    if (!m) {
        set_error("numa_mesh_create: out of host memory");
        return NUMA_ENOMEM;
    }
    m->d = *d;
    int32_t rc;
    try {
        rc = numa::build_mesh(*m);
    } catch (const std::bad_alloc &) {
        set_error("numa_mesh_create: out of host memory");
        rc = NUMA_ENOMEM;
    }
    if (rc != NUMA_OK) {
        delete m;
        return rc;
    }
    *out = m;
    return NUMA_OK;
}

static void drop_step_graph(numa_mesh_t m)
{
    if (m->step_exec) (void)hipGraphExecDestroy(m->step_exec);
    if (m->step_graph) (void)hipGraphDestroy(m->step_graph);
    m->step_exec = nullptr;
    m->step_graph = nullptr;
}

int32_t numa_mesh_destroy(numa_mesh_t m)
{
    if (m) {
        for (hipEvent_t e : m->ev_pool) (void)hipEventDestroy(e);
        drop_step_graph(m);
        if (m->cap_stream) (void)hipStreamDestroy(m->cap_stream);
    }
    delete m;
    return NUMA_OK;
}

int32_t numa_mesh_info(numa_mesh_t m, int64_t *n_elem, int64_t *n_local, int64_t *n_unique, int64_t *n_horiz,
                       int64_t *n_levels)
{
    if (!m) {
        set_error("numa_mesh_info: null mesh handle");
        return NUMA_EINVAL;
    }
    if (n_elem) *n_elem = m->ne;
    if (n_local) *n_local = m->nl;
    if (n_unique) *n_unique = m->nu;
    if (n_horiz) *n_horiz = m->nh;
    if (n_levels) *n_levels = m->nk;
    return NUMA_OK;
}

int32_t numa_mesh_gather_map(numa_mesh_t m, int32_t *host_out)
{
    if (!m || !host_out) {
        set_error("numa_mesh_gather_map: null argument");
        return NUMA_EINVAL;
    }
    std::memcpy(host_out, m->G.data(), sizeof(int32_t) * m->nl);
    return NUMA_OK;
}

int32_t numa_mesh_workspace_bytes(numa_mesh_t m, int32_t prec_mask, uint64_t *bytes)
{
    if (!m || !bytes) {
        set_error("numa_mesh_workspace_bytes: null argument");
        return NUMA_EINVAL;
    }
    *bytes = numa::layout_workspace(*m, prec_mask, nullptr);
    return NUMA_OK;
}

int32_t numa_mesh_attach_workspace(numa_mesh_t m, void *dev_ptr, uint64_t bytes, int32_t prec_mask)
{
    if (!m || !dev_ptr) {
        set_error("numa_mesh_attach_workspace: null argument");
        return NUMA_EINVAL;
    }
    if (reinterpret_cast<uintptr_t>(dev_ptr) % 256) {
        set_error("numa_mesh_attach_workspace: workspace must be 256-byte aligned");
        return NUMA_EINVAL;
    }
    if ((prec_mask & NUMA_WS_LEAN) && !numa::box_batchable(*m)) {
        set_error("numa_mesh_attach_workspace: NUMA_WS_LEAN needs a box mesh whose x element count fits the "
                  "batched finish");
        return NUMA_EUNSUPPORTED;
    }
    uint64_t need = numa::layout_workspace(*m, prec_mask, nullptr);
    if (bytes < need) {
        set_error("numa_mesh_attach_workspace: %llu bytes given, %llu needed", (unsigned long long)bytes,
                  (unsigned long long)need);
        return NUMA_ENOMEM;
    }
    m->ws = static_cast<char *>(dev_ptr);
    ++m->gen;
    m->ws_bytes = bytes;
    m->prec_mask = prec_mask | 1;
    numa::layout_workspace(*m, m->prec_mask, m->ws);
    m->uploaded = false;
    m->geom = false;
    m->imex_ok = false;
    return NUMA_OK;
}

int32_t numa_mesh_set_metric(numa_mesh_t m, int32_t mode)
{
    if (!m) {
        set_error("numa_mesh_set_metric: null mesh handle");
        return NUMA_EINVAL;
    }
    if (mode != NUMA_METRIC_STORED && mode != NUMA_METRIC_RECOMPUTE) {
        set_error("numa_mesh_set_metric: unknown mode %d", mode);
        return NUMA_EINVAL;
    }
    m->metric_mode = mode;
    ++m->gen;
    return NUMA_OK;
}

int32_t numa_mesh_set_stage(numa_mesh_t m, int32_t mode)
{
    if (!m) {
        set_error("numa_mesh_set_stage: null mesh handle");
        return NUMA_EINVAL;
    }
    if (mode != NUMA_STAGE_GATHER && mode != NUMA_STAGE_BLOCK && mode != NUMA_STAGE_COLOUR &&
        mode != NUMA_STAGE_SPLIT && mode != NUMA_STAGE_AUTO) {
        set_error("numa_mesh_set_stage: unknown mode %d", mode);
        return NUMA_EINVAL;
    }
    m->stage_mode = mode;
    ++m->gen;
    return NUMA_OK;
}

int32_t numa_geometry(numa_mesh_t m, const numa_phys *ph, void *stream)
{
    if (!m || !ph) {
        set_error("numa_geometry: null argument");
        return NUMA_EINVAL;
    }
    if (!m->ws) {
        set_error("numa_geometry: no workspace attached");
        return NUMA_ENOMEM;
    }
    if (!(ph->cp > ph->R && ph->R > 0 && ph->p0 > 0 && ph->T0 > 0 && ph->g0 >= 0)) {
        set_error("numa_geometry: invalid physical constants");
        return NUMA_EINVAL;
    }
    if (m->d.kind == NUMA_MESH_BOX && ph->g0 * m->d.extent[2] >= ph->cp * ph->T0) {
        set_error("numa_geometry: the isentropic reference reaches zero pressure below the model top");
        return NUMA_EINVAL;
    }
    m->ph = *ph;
    m->gamma = ph->cp / (ph->cp - ph->R);
    int32_t rc = numa::launch_geometry(*m, as_stream(stream));
    m->geom = rc == NUMA_OK;
    ++m->gen;
    m->imex_ok = false;  // the reference state may have changed
    return rc;
}

int32_t numa_export(numa_mesh_t m, int32_t what, void *dev_out, void *stream)
{
    int32_t rc = need_ready(m, "numa_export");
    if (rc) return rc;
    if (!dev_out) {
        set_error("numa_export: null output");
        return NUMA_EINVAL;
    }
    return numa::launch_export(*m, what, dev_out, as_stream(stream));
}

int32_t numa_init_state(numa_mesh_t m, const numa_ic *ic, const double *noise, double *q, void *stream)
{
    int32_t rc = need_ready(m, "numa_init_state");
    if (rc) return rc;
    if (!ic || !q) {
        set_error("numa_init_state: null argument");
        return NUMA_EINVAL;
    }
    if (ic->kind < 0 || ic->kind > 2 || (ic->kind == 2 && m->d.kind != NUMA_MESH_SHELL)) {
        set_error("numa_init_state: initial-condition kind %d not valid for this mesh", ic->kind);
        return NUMA_EINVAL;
    }
    if (ic->kind != 0 && !(ic->radius > 0) ) {
        set_error("numa_init_state: radius must be positive");
        return NUMA_EINVAL;
    }
    if (ic->kind == 2 && !(ic->lz > 0)) {
        set_error("numa_init_state: lz must be positive");
        return NUMA_EINVAL;
    }
    return numa::launch_init_state(*m, *ic, noise, q, as_stream(stream));
}

int32_t numa_rhs(numa_mesh_t m, int32_t prec, const double *q, double *c_elem, void *stream)
{
    int32_t rc = need_ready(m, "numa_rhs");
    if (rc) return rc;
    if ((rc = need_full(m, "numa_rhs"))) return rc;
    if ((rc = check_prec(m, prec, "numa_rhs"))) return rc;
    if (!q || !c_elem) {
        set_error("numa_rhs: null argument");
        return NUMA_EINVAL;
    }
    return numa::launch_rhs(*m, prec, q, c_elem, as_stream(stream));
}

int32_t numa_dss(numa_mesh_t m, int32_t nvar, const double *c_elem, double *out, int32_t flags, void *stream)
{
    int32_t rc = need_ready(m, "numa_dss");
    if (rc) return rc;
    if ((rc = need_full(m, "numa_dss"))) return rc;
    if (!c_elem || !out || nvar < 1) {
        set_error("numa_dss: null argument or nvar < 1");
        return NUMA_EINVAL;
    }
    if (flags & ~(NUMA_DSS_MASS | NUMA_DSS_NOFLUX)) {
        set_error("numa_dss: unknown flags 0x%x", flags);
        return NUMA_EINVAL;
    }
    if ((flags & NUMA_DSS_NOFLUX) && nvar != 5) {
        set_error("numa_dss: NUMA_DSS_NOFLUX needs nvar == 5");
        return NUMA_EINVAL;
    }
    return numa::launch_dss(*m, nvar, c_elem, out, flags, as_stream(stream));
}

static bool filter_params_ok(const char *fn, double filter_order, int32_t cutoff)
{
    if (!(filter_order > 0.0) || !std::isfinite(filter_order) || cutoff < 0) {
        set_error("%s: filter order must be finite and > 0 and the cutoff >= 0 (got %g, %d)", fn, filter_order,
                  cutoff);
        return false;
    }
    return true;
}

int32_t numa_filter_matrix(int32_t order, double filter_order, int32_t cutoff, double *F)
{
    double xi[numa::kMaxP], w[numa::kMaxP], D[numa::kMaxP * numa::kMaxP];
    if (!F) {
        set_error("numa_filter_matrix: null output");
        return NUMA_EINVAL;
    }
    if (!numa::gll(order, xi, w, D)) {
        set_error("numa_filter_matrix: order %d outside 1..8", order);
        return NUMA_EINVAL;
    }
    if (!filter_params_ok("numa_filter_matrix", filter_order, cutoff)) return NUMA_EINVAL;
    numa::filter_matrix(order, xi, w, filter_order, cutoff, F);
    return NUMA_OK;
}

int32_t numa_mesh_set_filter(numa_mesh_t m, int32_t enable, double filter_order, int32_t cutoff)
{
    if (!m) {
        set_error("numa_mesh_set_filter: null mesh handle");
        return NUMA_EINVAL;
    }
    if (enable && !filter_params_ok("numa_mesh_set_filter", filter_order, cutoff)) return NUMA_EINVAL;
    m->filter_on = enable != 0;
    ++m->gen;
    m->filter_order = enable ? filter_order : 0.0;
    m->filter_cutoff = enable ? cutoff : 0;
    return NUMA_OK;
}

int32_t numa_filter(numa_mesh_t m, double filter_order, int32_t cutoff, double *q, void *stream)
{
    int32_t rc = need_ready(m, "numa_filter");
    if (rc) return rc;
    if ((rc = need_full(m, "numa_filter"))) return rc;
    if (!q) {
        set_error("numa_filter: null state");
        return NUMA_EINVAL;
    }
    if (!filter_params_ok("numa_filter", filter_order, cutoff)) return NUMA_EINVAL;
    return numa::launch_filter(*m, filter_order, cutoff, q, as_stream(stream));
}

int32_t numa_rk_stage(numa_mesh_t m, int32_t stage, double dt, const double *qn, const double *qs, const double *r,
                      double *qout, void *stream)
{
    int32_t rc = need_ready(m, "numa_rk_stage");
    if (rc) return rc;
    if (stage < 0 || stage > 2) {
        set_error("numa_rk_stage: stage %d outside 0..2", stage);
        return NUMA_EINVAL;
    }
    if (!qs || !r || !qout || (stage > 0 && !qn)) {
        set_error("numa_rk_stage: null argument");
        return NUMA_EINVAL;
    }
    return numa::launch_rk_stage(*m, stage, dt, qn, qs, r, qout, as_stream(stream));
}

// event bracket around a group of launches when the mesh is profiling
static int32_t mark(numa_mesh_t m, std::vector<std::pair<int, int>> &log, bool begin, hipStream_t s)
{
    if (!m || !m->profiling) return NUMA_OK;
    if (m->ev_used == m->ev_pool.size()) {
        hipEvent_t e;
        NUMA_HIP(hipEventCreate(&e));
        m->ev_pool.push_back(e);
    }
    int id = (int)m->ev_used++;
    NUMA_HIP(hipEventRecord(m->ev_pool[id], s));
    if (begin) log.push_back({id, -1});
    else log.back().second = id;
    return NUMA_OK;
}

// one fused stage of a batch: element kernels then finish kernels; events are
// recorded on the first item's mesh when it is profiling
static int32_t run_batch_stage(const numa::StepItem *items, int n, int32_t prec, hipStream_t s)
{
    numa_mesh_t m0 = static_cast<numa_mesh_t>(const_cast<Mesh *>(items[0].mesh));
    int32_t rc;
    if ((rc = mark(m0, m0->ev_elem, true, s))) return rc;
    if ((rc = numa::launch_batch_stage(items, n, prec, 0, s))) return rc;
    if ((rc = mark(m0, m0->ev_elem, false, s))) return rc;
    if ((rc = mark(m0, m0->ev_fin, true, s))) return rc;
    if ((rc = numa::launch_batch_stage(items, n, prec, 1, s))) return rc;
    return mark(m0, m0->ev_fin, false, s);
}

// one fused stage of a single mesh through the general kernels (shell, or a
// box whose x extent does not fit the batched finish)
static int32_t run_stage(numa_mesh_t m, int32_t prec, const numa::StageCoef &c, const double *qn, const double *qs,
                         double *qout, hipStream_t s)
{
    int32_t rc;
    if ((rc = mark(m, m->ev_elem, true, s))) return rc;
    if ((rc = numa::launch_stage_elements(*m, prec, c, qs, s))) return rc;
    if ((rc = mark(m, m->ev_elem, false, s))) return rc;
    if ((rc = mark(m, m->ev_fin, true, s))) return rc;
    if ((rc = numa::launch_stage_finish(*m, prec, c, qn, qs, qout, s))) return rc;
    return mark(m, m->ev_fin, false, s);
}

// the filter at the end of a step (Code example 1), when set on the mesh
static int32_t run_filter(numa_mesh_t m, double *q, hipStream_t s)
{
    if (!m->filter_on) return NUMA_OK;
    return numa::launch_filter(*m, m->filter_order, m->filter_cutoff, q, s);
}

// The stages of one step in Shu-Osher form.  Buffers: 0 = q (u_0 = q^n at the
// start, q^{n+1} at the end), 1 and 2 = stage scratch.  A stage evaluates the
// right-hand side on buffer `in` and writes a q_ref + b (u_in + (beta/b) dt R)
// to `out` (ref is not read when a = 0).  `out` may equal `in`: the finish is
// pointwise and the element kernel has read `in` before it runs.
struct StagePlan {
    int in, ref, out;
    double a, b, beta;
};
// SSP-RK3 (Shu-Osher): (a, b) = (0, 1), (3/4, 1/4), (1/3, 2/3), beta = b.
// No stage writes its own input: the fused block stage finishes nodes while
// other workgroups still gather the input state.
static const StagePlan kSsp33[3] = {
    {0, 0, 1, 0.0, 1.0, 1.0}, {1, 0, 2, 0.75, 0.25, 0.25}, {2, 0, 0, 1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0}};
// Five-stage third-order SSP Runge-Kutta (Spiteri and Ruuth, SIAM J. Numer.
// Anal. 40(2), 2002), the paper's explicit scheme class (Sec. "Time
// Discretization": five stages, third order):
//   u1 = u0 + b10 dt L(u0),  u2 = u1 + b21 dt L(u1),
//   u3 = a30 u0 + a32 u2 + b32 dt L(u2),  u4 = a40 u0 + a43 u3 + b43 dt L(u3),
//   u5 = a52 u2 + a54 u4 + b54 dt L(u4).
// Buffer 1 holds u1, u3, u4; buffer 2 holds u2 until the last stage.
static const StagePlan kSsp53[5] = {
    {0, 0, 1, 0.0, 1.0, 0.377268915331368},
    {1, 0, 2, 0.0, 1.0, 0.377268915331368},
    {2, 0, 1, 0.355909775063327, 0.644090224936674, 0.242995220537396},
    {1, 0, 1, 0.367933791638137, 0.632066208361863, 0.238458932846290},
    {1, 2, 0, 0.237593836598569, 0.762406163401431, 0.287632146308408}};

static const StagePlan *stage_plan(int integrator, int *nstages)
{
    *nstages = integrator == NUMA_RK_SSP53 ? 5 : 3;
    return integrator == NUMA_RK_SSP53 ? kSsp53 : kSsp33;
}

static numa::StageCoef stage_coef(const StagePlan &p, double dt)
{
    // SSP-RK3 keeps cdt = dt exactly (beta = b)
    return numa::StageCoef{p.a, p.b, p.beta == p.b ? dt : (p.beta / p.b) * dt};
}

int32_t numa_mesh_set_integrator(numa_mesh_t m, int32_t integrator)
{
    if (!m) {
        set_error("numa_mesh_set_integrator: null mesh handle");
        return NUMA_EINVAL;
    }
    if (integrator != NUMA_RK_SSP33 && integrator != NUMA_RK_SSP53) {
        set_error("numa_mesh_set_integrator: unknown integrator %d", integrator);
        return NUMA_EINVAL;
    }
    m->integrator = integrator;
    ++m->gen;
    return NUMA_OK;
}

// the launches of one step of the mesh's integrator (and its filter) on q
static int32_t enqueue_step(numa_mesh_t m, int32_t prec, double dt, double *q, hipStream_t s)
{
    double *buf[3] = {q, m->dv.qs, m->dv.qs2};
    int ns;
    const StagePlan *plan = stage_plan(m->integrator, &ns);
    const bool batched = numa::stage_batched(*m, prec);
    void *ev = m->dv.ev64;  // FP64-sized: element contributions of either precision, or an FP64 accumulator
    int32_t rc;
    for (int k = 0; k < ns; ++k) {
        const StagePlan &p = plan[k];
        const numa::StageCoef c = stage_coef(p, dt);
        if (batched) {
            numa::StepItem it = {m, buf[p.ref], buf[p.in], buf[p.out], ev, c};
            rc = run_batch_stage(&it, 1, prec, s);
        } else {
            rc = run_stage(m, prec, c, buf[p.ref], buf[p.in], buf[p.out], s);
        }
        if (rc) return rc;
    }
    return run_filter(m, q, s);
}

// the captured step for (prec, dt, q) under the mesh's current settings,
// recorded on the mesh's own capture stream when it is not cached
static int32_t step_exec(numa_mesh_t m, int32_t prec, double dt, double *q, hipGraphExec_t *out)
{
    if (m->step_exec && m->g_prec == prec && m->g_dt == dt && m->g_q == q && m->g_gen == m->gen) {
        *out = m->step_exec;
        return NUMA_OK;
    }
    drop_step_graph(m);
    if (!m->cap_stream) NUMA_HIP(hipStreamCreateWithFlags(&m->cap_stream, hipStreamNonBlocking));
    NUMA_HIP(hipStreamBeginCapture(m->cap_stream, hipStreamCaptureModeThreadLocal));
    int32_t rc = enqueue_step(m, prec, dt, q, m->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(m->cap_stream, &g);
    if (rc != NUMA_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        if (rc == NUMA_OK) set_error("numa_step: hipStreamEndCapture failed: %s", hipGetErrorString(e));
        return rc != NUMA_OK ? rc : NUMA_EDEVICE;
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        set_error("numa_step: hipGraphInstantiate failed: %s", hipGetErrorString(e));
        return NUMA_EDEVICE;
    }
    m->step_graph = g;
    m->step_exec = x;
    m->g_prec = prec;
    m->g_dt = dt;
    m->g_q = q;
    m->g_gen = m->gen;
    *out = x;
    return NUMA_OK;
}

int32_t numa_step(numa_mesh_t m, int32_t prec, double dt, int32_t nsteps, double *q, void *stream)
{
    int32_t rc = need_ready(m, "numa_step");
    if (rc) return rc;
    if ((rc = need_full(m, "numa_step"))) return rc;
    if ((rc = check_prec(m, prec, "numa_step"))) return rc;
    if (!q || nsteps < 0) {
        set_error("numa_step: null state or negative step count");
        return NUMA_EINVAL;
    }
    if (nsteps == 0) return NUMA_OK;
    hipStream_t s = as_stream(stream);
    // replay the captured step unless the caller is capturing this stream
    // itself or the stage kernels are being timed one by one
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    NUMA_HIP(hipStreamIsCapturing(s, &cs));
    if (m->step_graphs && !m->profiling && cs == hipStreamCaptureStatusNone) {
        hipGraphExec_t x;
        if ((rc = step_exec(m, prec, dt, q, &x))) return rc;
        for (int n = 0; n < nsteps; ++n) NUMA_HIP(hipGraphLaunch(x, s));
        return NUMA_OK;
    }
    for (int n = 0; n < nsteps; ++n)
        if ((rc = enqueue_step(m, prec, dt, q, s))) return rc;
    return NUMA_OK;
}

int32_t numa_mesh_set_step_graph(numa_mesh_t m, int32_t enable)
{
    if (!m) {
        set_error("numa_mesh_set_step_graph: null mesh handle");
        return NUMA_EINVAL;
    }
    m->step_graphs = enable != 0;
    if (!m->step_graphs) drop_step_graph(m);
    return NUMA_OK;
}

int32_t numa_stage_rhs(numa_mesh_t m, int32_t prec, const double *q, double *r, void *stream)
{
    int32_t rc = need_ready(m, "numa_stage_rhs");
    if (rc) return rc;
    if ((rc = need_full(m, "numa_stage_rhs"))) return rc;
    if ((rc = check_prec(m, prec, "numa_stage_rhs"))) return rc;
    if (!q || !r) {
        set_error("numa_stage_rhs: null argument");
        return NUMA_EINVAL;
    }
    if (q == r) {
        set_error("numa_stage_rhs: r must not alias q");
        return NUMA_EINVAL;
    }
    hipStream_t s = as_stream(stream);
    // a stage whose update is q_out = 0 q_ref + 1 R (b = 0: no q_s term, so no
    // kernel folds q_s into the contributions): the summed, mass-weighted,
    // projected right-hand side itself
    const numa::StageCoef c{0.0, 0.0, 1.0};
    if (numa::stage_batched(*m, prec)) {
        void *ev = m->dv.ev64;  // FP64-sized: element contributions of either precision, or an FP64 accumulator
        numa::StepItem it = {m, q, q, r, ev, c};
        return run_batch_stage(&it, 1, prec, s);
    }
    return run_stage(m, prec, c, q, q, r, s);
}

int32_t numa_imex_step(numa_mesh_t m, int32_t prec, double dt, double ra, int32_t nsteps, double *qprev,
                       double *qcur, void *stream)
{
    int32_t rc = need_ready(m, "numa_imex_step");
    if (rc) return rc;
    if ((rc = need_full(m, "numa_imex_step"))) return rc;
    if ((rc = check_prec(m, prec, "numa_imex_step"))) return rc;
    if (!qprev || !qcur || qprev == qcur || nsteps < 0) {
        set_error("numa_imex_step: null or identical states, or negative step count");
        return NUMA_EINVAL;
    }
    if (!std::isfinite(dt) || !(ra >= 0.0 && ra < 1.0)) {
        set_error("numa_imex_step: dt must be finite and the Robert-Asselin coefficient in [0, 1)");
        return NUMA_EINVAL;
    }
    if (!m->walls) {
        set_error("numa_imex_step: the vertical correction needs no-flux walls (a box periodic in z has none)");
        return NUMA_EUNSUPPORTED;
    }
    if (numa::imex_lds_bytes(*m) > 65536) {
        set_error("numa_imex_step: %llu levels need more than 64 KB of LDS per vertical line",
                  (unsigned long long)m->nk);
        return NUMA_EUNSUPPORTED;
    }
    if (!m->dv.imexLU) {
        set_error("numa_imex_step: attach the workspace with NUMA_WS_IMEX for the line factors");
        return NUMA_ENOMEM;
    }
    hipStream_t s = as_stream(stream);
    if (!m->imex_ok || m->imex_dt != dt) {  // factors of I - dt V, once per dt
        if ((rc = numa::launch_imex_factor(*m, dt, s))) return rc;
        m->imex_dt = dt;
        m->imex_ok = true;
    }
    const numa::StageCoef c{1.0, 0.0, 2.0 * dt};  // q* = q^{n-1} + 2 dt L(q^n)
    void *ev = m->dv.ev64;  // FP64-sized: element contributions of either precision, or an FP64 accumulator
    for (int n = 0; n < nsteps; ++n) {
        if (numa::stage_batched(*m, prec)) {
            numa::StepItem it = {m, qprev, qcur, m->dv.qs, ev, c};
            rc = run_batch_stage(&it, 1, prec, s);
        } else {
            rc = run_stage(m, prec, c, qprev, qcur, m->dv.qs, s);
        }
        if (rc) return rc;
        if ((rc = numa::launch_imex_correction(*m, dt, ra, qprev, qcur, s))) return rc;
    }
    return NUMA_OK;
}

static uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

// the contribution scratch of a batch item: element contributions of the
// precision, the fused block stage's partial sums, or the colour passes' FP64
// accumulator [5][n_unique]
static uint64_t contribution_bytes(const Mesh &m, int32_t prec)
{
    const uint64_t ev = (prec == NUMA_PREC_MIXED ? 20ull : 40ull) * m.nl, acc = 40ull * m.nu;
    return align256(ev > acc ? ev : acc);
}

// batch-item scratch: stage state, contributions, second stage state
static uint64_t scratch_bytes(const Mesh &m, int32_t prec)
{
    return align256(40ull * m.nu) + contribution_bytes(m, prec) + align256(40ull * m.nu);
}

int32_t numa_step_scratch_bytes(numa_mesh_t m, int32_t prec, uint64_t *bytes)
{
    if (!m || !bytes) {
        set_error("numa_step_scratch_bytes: null argument");
        return NUMA_EINVAL;
    }
    *bytes = scratch_bytes(*m, prec);
    return NUMA_OK;
}

}  // extern "C"

// own_scratch: the items bring their scratch (numa_step_batch), else the
// library supplies it, the items' scratch fields must be empty and no mesh
// may be profiling (that creates events)
int32_t numa::check_batch(const numa_batch_item *items, int32_t n, int32_t prec, bool own_scratch, const char *fn)
{
    if (!items || n < 1) {
        set_error("%s: no items", fn);
        return NUMA_EINVAL;
    }
    for (int32_t k = 0; k < n; ++k) {
        numa_mesh_t m = items[k].mesh;
        int32_t rc = need_ready(m, fn);
        if (rc) return rc;
        if ((rc = check_prec(m, prec, fn))) return rc;
        if (!numa::stage_batched(*m, prec)) {
            set_error("%s: item %d: batched stages need a box mesh whose x element count fits the finish segment "
                      "(or NUMA_STAGE_SPLIT with the recomputed metric, N <= 4)", fn, k);
            return NUMA_EUNSUPPORTED;
        }
        if (m->N != items[0].mesh->N) {
            set_error("%s: item %d has order %d, item 0 has %d (one order per batch)", fn, k, m->N, items[0].mesh->N);
            return NUMA_EINVAL;
        }
        if (m->metric_mode != items[0].mesh->metric_mode) {
            set_error("%s: item %d uses another metric mode than item 0 (one mode per batch)", fn, k);
            return NUMA_EINVAL;
        }
        if (m->lean && m->metric_mode != NUMA_METRIC_RECOMPUTE) {
            set_error("%s: item %d: a lean workspace (NUMA_WS_LEAN) holds no stored metric: set "
                      "NUMA_METRIC_RECOMPUTE", fn, k);
            return NUMA_EINVAL;
        }
        if (m->lean && m->filter_on) {
            set_error("%s: item %d: the filter needs the contribution scratch a lean workspace does not hold", fn, k);
            return NUMA_ENOMEM;
        }
        if (m->integrator != items[0].mesh->integrator) {
            set_error("%s: item %d uses another integrator than item 0 (one integrator per batch)", fn, k);
            return NUMA_EINVAL;
        }
        if (!items[k].q) {
            set_error("%s: item %d: null state", fn, k);
            return NUMA_EINVAL;
        }
        if (!own_scratch) {
            if (items[k].scratch || items[k].scratch_bytes) {
                set_error("%s: item %d: the library supplies the scratch; pass NULL and 0", fn, k);
                return NUMA_EINVAL;
            }
            if (m->profiling) {  // the profile creates events as it goes
                set_error("%s: item %d: disable numa_profile on the items' meshes first", fn, k);
                return NUMA_EINVAL;
            }
        } else if (!items[k].scratch || reinterpret_cast<uintptr_t>(items[k].scratch) % 256) {
            set_error("%s: item %d: null scratch or scratch not 256-byte aligned", fn, k);
            return NUMA_EINVAL;
        } else if (items[k].scratch_bytes < scratch_bytes(*m, prec)) {
            set_error("%s: item %d: scratch of %llu bytes, the item needs %llu", fn, k,
                      (unsigned long long)items[k].scratch_bytes, (unsigned long long)scratch_bytes(*m, prec));
            return NUMA_ENOMEM;
        }
        for (int32_t j = 0; j < k; ++j)
            if (items[j].q == items[k].q || (own_scratch && items[j].scratch == items[k].scratch)) {
                set_error("%s: items %d and %d share a state or a scratch buffer", fn, j, k);
                return NUMA_EINVAL;
            }
    }
    return NUMA_OK;
}

uint64_t numa::batch_pool_bytes(const numa_batch_item *items, int32_t n, int32_t prec)
{
    uint64_t total = 0;
    for (int32_t k = 0; k < n; ++k) total += scratch_bytes(*items[k].mesh, prec);
    return total;
}

int numa::batch_stages(const numa_batch_item *items)
{
    int ns;
    (void)stage_plan(items[0].mesh->integrator, &ns);
    return ns;
}

// nsteps steps of a checked batch.  pool: null when each item brings its
// scratch, else the items' scratch lies one after another in pool (each
// numa_step_scratch_bytes, a multiple of 256).  st: room for the stages of
// the integrator times n stage items.
int32_t numa::run_step_batch(const numa_batch_item *items, int32_t n, int32_t prec, int32_t nsteps, char *pool,
                             StepItem *st, hipStream_t s)
{
    int ns;
    const StagePlan *plan = stage_plan(items[0].mesh->integrator, &ns);
    for (int32_t k = 0; k < n; ++k) {
        const Mesh *m = items[k].mesh;
        char *scr = pool ? pool : static_cast<char *>(items[k].scratch);
        if (pool) pool += scratch_bytes(*m, prec);
        const uint64_t evb = contribution_bytes(*m, prec);
        double *buf[3] = {items[k].q, reinterpret_cast<double *>(scr),
                          reinterpret_cast<double *>(scr + align256(40ull * m->nu) + evb)};
        void *ev = scr + align256(40ull * m->nu);
        for (int j = 0; j < ns; ++j) {
            const StagePlan &p = plan[j];
            st[(size_t)j * n + k] = {m, buf[p.ref], buf[p.in], buf[p.out], ev, stage_coef(p, items[k].dt),
                                     items[k].nonfinite};
        }
    }
    int32_t rc;
    for (int32_t step = 0; step < nsteps; ++step) {
        for (int j = 0; j < ns; ++j)
            if ((rc = run_batch_stage(&st[(size_t)j * n], n, prec, s))) return rc;
        for (int32_t k = 0; k < n; ++k)  // one after another: items may share a mesh's scratch
            if ((rc = run_filter(items[k].mesh, items[k].q, s))) return rc;
    }
    return NUMA_OK;
}

extern "C" {

int32_t numa_step_batch(const numa_batch_item *items, int32_t n, int32_t prec, int32_t nsteps, void *stream)
{
    int32_t rc = numa::check_batch(items, n, prec, true, "numa_step_batch");
    if (rc) return rc;
    if (nsteps < 0) {
        set_error("numa_step_batch: negative step count");
        return NUMA_EINVAL;
    }
    std::vector<numa::StepItem> st((size_t)numa::batch_stages(items) * n);
    return numa::run_step_batch(items, n, prec, nsteps, nullptr, st.data(), as_stream(stream));
}

int32_t numa_batch_capture(const numa_batch_item *items, int32_t n, int32_t prec, int32_t nsteps, void *stream,
                           numa_graph_t *out)
{
    if (!out) {
        set_error("numa_batch_capture: null output");
        return NUMA_EINVAL;
    }
    *out = nullptr;
    int32_t rc = numa::check_batch(items, n, prec, true, "numa_batch_capture");
    if (rc) return rc;
    if (!stream) {
        set_error("numa_batch_capture: capture needs a non-default stream");
        return NUMA_EINVAL;
    }
    for (int32_t k = 0; k < n; ++k)
        if (items[k].mesh->profiling) {
            set_error("numa_batch_capture: disable numa_profile on the items' meshes first");
            return NUMA_EINVAL;
        }
    hipStream_t s = as_stream(stream);
    NUMA_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    rc = numa_step_batch(items, n, prec, nsteps, stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (rc != NUMA_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) {
        set_error("numa_batch_capture: hipStreamEndCapture failed: %s", hipGetErrorString(e));
        return NUMA_EDEVICE;
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        set_error("numa_batch_capture: hipGraphInstantiate failed: %s", hipGetErrorString(e));
        return NUMA_EDEVICE;
    }
    numa_graph *h = new (std::nothrow) numa_graph{g, x};
    if (!h) {
        (void)hipGraphExecDestroy(x);
        (void)hipGraphDestroy(g);
        set_error("numa_batch_capture: out of host memory");
        return NUMA_ENOMEM;
    }
    *out = h;
    return NUMA_OK;
}

int32_t numa_graph_launch(numa_graph_t g, void *stream)
{
    if (!g) {
        set_error("numa_graph_launch: null graph");
        return NUMA_EINVAL;
    }
    NUMA_HIP(hipGraphLaunch(g->exec, as_stream(stream)));
    return NUMA_OK;
}

int32_t numa_graph_destroy(numa_graph_t g)
{
    if (!g) return NUMA_OK;
    hipError_t e1 = hipGraphExecDestroy(g->exec), e2 = hipGraphDestroy(g->graph);
    delete g;
    if (e1 != hipSuccess || e2 != hipSuccess) {
        set_error("numa_graph_destroy: %s", hipGetErrorString(e1 != hipSuccess ? e1 : e2));
        return NUMA_EDEVICE;
    }
    return NUMA_OK;
}

int32_t numa_profile(numa_mesh_t m, int32_t enable)
{
    if (!m) {
        set_error("numa_profile: null mesh handle");
        return NUMA_EINVAL;
    }
    m->profiling = enable != 0;
    m->ev_elem.clear();
    m->ev_fin.clear();
    m->ev_used = 0;
    return NUMA_OK;
}

int32_t numa_profile_read(numa_mesh_t m, double *out)
{
    if (!m || !out) {
        set_error("numa_profile_read: null argument");
        return NUMA_EINVAL;
    }
    const std::vector<std::pair<int, int>> *logs[2] = {&m->ev_elem, &m->ev_fin};
    for (int k = 0; k < 2; ++k) {
        double total = 0.0;
        int n = 0;
        for (auto &pr : *logs[k]) {
            if (pr.second < 0) continue;
            NUMA_HIP(hipEventSynchronize(m->ev_pool[pr.second]));
            float ms = 0.0f;
            NUMA_HIP(hipEventElapsedTime(&ms, m->ev_pool[pr.first], m->ev_pool[pr.second]));
            total += ms;
            ++n;
        }
        out[2 * k] = total;
        out[2 * k + 1] = n;
    }
    return NUMA_OK;
}

}  // extern "C"
