// C-ABI entry points of libnuma (declared in include/numa.h): argument
// checking, error reporting, workspace binding and the stage sequencing of
// numa_step.  All arithmetic of the path runs in the HIP kernels.
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

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

int32_t numa_mesh_destroy(numa_mesh_t m)
{
    if (m)
        for (hipEvent_t e : m->ev_pool) (void)hipEventDestroy(e);
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
    uint64_t need = numa::layout_workspace(*m, prec_mask, nullptr);
    if (bytes < need) {
        set_error("numa_mesh_attach_workspace: %llu bytes given, %llu needed", (unsigned long long)bytes,
                  (unsigned long long)need);
        return NUMA_ENOMEM;
    }
    m->ws = static_cast<char *>(dev_ptr);
    m->ws_bytes = bytes;
    m->prec_mask = prec_mask | 1;
    numa::layout_workspace(*m, m->prec_mask, m->ws);
    m->uploaded = false;
    m->geom = false;
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

// one fused stage: element kernel then finish kernel, optionally bracketed by events
static int32_t run_stage(numa_mesh_t m, int32_t prec, int32_t stage, double dt, const double *qn, const double *qs,
                         double *qout, hipStream_t s)
{
    int32_t rc;
    auto mark = [&](std::vector<std::pair<int, int>> &log, bool begin) -> int32_t {
        if (!m->profiling) return NUMA_OK;
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
    };
    if ((rc = mark(m->ev_elem, true))) return rc;
    if ((rc = numa::launch_stage_elements(*m, prec, stage, dt, qn, qs, qout, s))) return rc;
    if ((rc = mark(m->ev_elem, false))) return rc;
    if ((rc = mark(m->ev_fin, true))) return rc;
    if ((rc = numa::launch_stage_finish(*m, prec, stage, dt, qn, qs, qout, s))) return rc;
    return mark(m->ev_fin, false);
}

int32_t numa_step(numa_mesh_t m, int32_t prec, double dt, int32_t nsteps, double *q, void *stream)
{
    int32_t rc = need_ready(m, "numa_step");
    if (rc) return rc;
    if ((rc = check_prec(m, prec, "numa_step"))) return rc;
    if (!q || nsteps < 0) {
        set_error("numa_step: null state or negative step count");
        return NUMA_EINVAL;
    }
    hipStream_t s = as_stream(stream);
    double *qs = m->dv.qs;
    for (int n = 0; n < nsteps; ++n) {
        if ((rc = run_stage(m, prec, 0, dt, q, q, qs, s))) return rc;
        if ((rc = run_stage(m, prec, 1, dt, q, qs, qs, s))) return rc;
        if ((rc = run_stage(m, prec, 2, dt, q, qs, q, s))) return rc;
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
