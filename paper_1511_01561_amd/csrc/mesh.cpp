// Host side of libnuma: GLL basis and the mesh numbering.
//
// The paper builds its meshes with p4est/p6est and converts the adjacency into
// a lookup table that also enumerates the CG nodes (Sec. "Mesh generation and
// load balancing").  Here the two structured meshes of the workloads (a box
// and a cubed-sphere shell) are numbered directly: one unique id per grid
// point (CG storage), an element -> unique gather map and its inverse.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "numa_internal.h"

namespace numa {

// Legendre P_N and its first two derivatives at x (three-term recurrence).
static void legendre3(int N, double x, double &p, double &dp, double &d2p)
{
    double pm = 1.0, pc = x;
    if (N == 0) { p = 1.0; dp = 0.0; d2p = 0.0; return; }
    for (int n = 2; n <= N; ++n) {
        double pn = ((2 * n - 1) * x * pc - (n - 1) * pm) / n;
        pm = pc;
        pc = pn;
    }
    p = pc;
    // (1 - x^2) P' = N (P_{N-1} - x P_N);  (1 - x^2) P'' = 2 x P' - N (N+1) P
    double s = 1.0 - x * x;
    dp = N * (pm - x * pc) / s;
    d2p = (2.0 * x * dp - N * (N + 1.0) * pc) / s;
}

// GLL nodes: -1, 1 and the zeros of P_N' (Newton with P_N''); weights
// 2/(N(N+1)P_N^2); derivative matrix by barycentric Lagrange differentiation,
// diagonal from the zero row sum of the derivative of a constant.
bool gll(int N, double *xi, double *w, double *D)
{
    if (N < 1 || N > kMaxP - 1) return false;
    const int P = N + 1;
    const double pi = 3.14159265358979323846;
    xi[0] = -1.0;
    xi[N] = 1.0;
    for (int i = 1; i <= N / 2; ++i) {
        double x = -std::cos(pi * i / N);
        for (int it = 0; it < 60; ++it) {
            double p, dp, d2p;
            legendre3(N, x, p, dp, d2p);
            double dx = dp / d2p;
            x -= dx;
            if (std::fabs(dx) <= 1e-17) break;
        }
        xi[i] = x;
        xi[N - i] = -x;
    }
    if (N % 2 == 0) xi[N / 2] = 0.0;
    for (int i = 0; i < P; ++i) {
        double p, dp, d2p;
        if (i == 0 || i == N) {
            p = (i == 0 && (N % 2)) ? -1.0 : 1.0;
        } else {
            legendre3(N, xi[i], p, dp, d2p);
        }
        w[i] = 2.0 / (N * (N + 1.0) * p * p);
    }
    // barycentric weights lambda_m = 1 / prod_{n != m} (x_m - x_n)
    double lam[kMaxP];
    for (int m = 0; m < P; ++m) {
        double prod = 1.0;
        for (int n = 0; n < P; ++n)
            if (n != m) prod *= (xi[m] - xi[n]);
        lam[m] = 1.0 / prod;
    }
    for (int i = 0; i < P; ++i) {
        double diag = 0.0;
        for (int m = 0; m < P; ++m) {
            if (m == i) continue;
            double v = (lam[m] / lam[i]) / (xi[i] - xi[m]);
            D[i * P + m] = v;
            diag -= v;
        }
        D[i * P + i] = diag;
    }
    return true;
}

// Cube-surface lattice point of face f at face coordinates (s, t), outward
// right-handed (s, t, radial):
//   f0 (L,s,t) f1 (L-s,L,t) f2 (0,L-s,t) f3 (s,0,t) f4 (s,t,L) f5 (t,s,0).
static inline void face_point(int f, int L, int s, int t, int p[3])
{
    static const int sel[6][3][3] = {
        // for each face and each of X,Y,Z: coefficients {const*L, s, t} in a tiny table
        {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}},
        {{1, -1, 0}, {1, 0, 0}, {0, 0, 1}},
        {{0, 0, 0}, {1, -1, 0}, {0, 0, 1}},
        {{0, 1, 0}, {0, 0, 0}, {0, 0, 1}},
        {{0, 1, 0}, {0, 0, 1}, {1, 0, 0}},
        {{0, 0, 1}, {0, 1, 0}, {0, 0, 0}},
    };
    for (int a = 0; a < 3; ++a) p[a] = sel[f][a][0] * L + sel[f][a][1] * s + sel[f][a][2] * t;
}

int32_t build_mesh(Mesh &m)
{
    const numa_mesh_desc &d = m.d;
    const int N = d.order;
    if (N < 1 || N > 8) {
        set_error("order %d outside 1..8", N);
        return NUMA_EINVAL;
    }
    m.N = N;
    m.P = N + 1;
    m.np = m.P * m.P * m.P;
    gll(N, m.xi, m.w, m.D);
    const int P = m.P, np = m.np;
    if (d.kind == NUMA_MESH_BOX) {
        for (int a = 0; a < 3; ++a)
            if (d.ne[a] < 1) { set_error("box: ne[%d] = %d < 1", a, d.ne[a]); return NUMA_EINVAL; }
        if (!d.periodic[0] || !d.periodic[1]) {
            set_error("box: x and y must be periodic");
            return NUMA_EINVAL;
        }
        for (int a = 0; a < 3; ++a)
            if (d.periodic[a] && d.ne[a] < 2) {
                set_error("box: periodic direction %d needs at least 2 elements", a);
                return NUMA_EINVAL;
            }
        if (!(d.extent[0] > 0 && d.extent[1] > 0 && d.extent[2] > 0)) {
            set_error("box: extents must be positive");
            return NUMA_EINVAL;
        }
        const int64_t nx = d.ne[0], ny = d.ne[1], nz = d.ne[2];
        m.ni = nx * N;
        m.nj = ny * N;
        m.nk = d.periodic[2] ? nz * N : nz * N + 1;
        m.walls = !d.periodic[2];
        m.ne = nx * ny * nz;
        m.nh = m.ni * m.nj;
        m.nu = m.nh * m.nk;
    } else if (d.kind == NUMA_MESH_SHELL) {
        if (d.ne[0] < 1 || d.ne[2] < 1) { set_error("shell: ne must be >= 1"); return NUMA_EINVAL; }
        if (!(d.extent[0] > 0 && d.extent[2] > 0)) { set_error("shell: radius and depth must be positive"); return NUMA_EINVAL; }
        const int64_t L = (int64_t)d.ne[0] * N;
        m.ne = 6 * (int64_t)d.ne[0] * d.ne[0] * d.ne[2];
        m.nh = 6 * L * L + 2;
        m.nk = (int64_t)d.ne[2] * N + 1;
        m.nu = m.nh * m.nk;
        m.walls = true;
    } else {
        set_error("unknown mesh kind %d", d.kind);
        return NUMA_EINVAL;
    }
    m.nl = m.ne * np;
    if (m.nl >= (int64_t(1) << 31) || m.nu >= (int64_t(1) << 31)) {
        set_error("mesh too large for 32-bit node indices");
        return NUMA_EUNSUPPORTED;
    }
    m.G.resize(m.nl);
    if (d.kind == NUMA_MESH_BOX) {
        const int nx = d.ne[0], ny = d.ne[1], nz = d.ne[2];
        int64_t e = 0;
        for (int ez = 0; ez < nz; ++ez)
            for (int ey = 0; ey < ny; ++ey)
                for (int ex = 0; ex < nx; ++ex, ++e) {
                    int32_t *g = m.G.data() + e * np;
                    for (int k = 0; k < P; ++k) {
                        int64_t gk = (int64_t)ez * N + k;
                        if (gk == m.nk) gk = 0;  // periodic z wraps the top layer
                        for (int j = 0; j < P; ++j) {
                            int64_t gj = (int64_t)ey * N + j;
                            if (gj == m.nj) gj = 0;
                            for (int i = 0; i < P; ++i) {
                                int64_t gi = (int64_t)ex * N + i;
                                if (gi == m.ni) gi = 0;
                                *g++ = (int32_t)(gi + m.ni * (gj + m.nj * gk));
                            }
                        }
                    }
                }
    } else {
        const int ne1 = d.ne[0], nz = d.ne[2];
        const int L = ne1 * N;
        const int64_t L1 = L + 1;
        // first-occurrence numbering of the surface lattice points (face, t, s order)
        std::vector<int32_t> hid(L1 * L1 * L1, -1);
        m.hlat.assign(3 * m.nh, 0);
        int32_t next = 0;
        for (int f = 0; f < 6; ++f)
            for (int t = 0; t <= L; ++t)
                for (int s = 0; s <= L; ++s) {
                    int p[3];
                    face_point(f, L, s, t, p);
                    int32_t &h = hid[p[0] + L1 * (p[1] + L1 * p[2])];
                    if (h < 0) {
                        h = next++;
                        m.hlat[3 * h] = p[0];
                        m.hlat[3 * h + 1] = p[1];
                        m.hlat[3 * h + 2] = p[2];
                    }
                }
        if (next != m.nh) {
            set_error("internal: shell lattice count %d != %lld", next, (long long)m.nh);
            return NUMA_EINVAL;
        }
        int64_t e = 0;
        for (int ez = 0; ez < nz; ++ez)
            for (int f = 0; f < 6; ++f)
                for (int ey = 0; ey < ne1; ++ey)
                    for (int ex = 0; ex < ne1; ++ex, ++e) {
                        int32_t *g = m.G.data() + e * np;
                        for (int k = 0; k < P; ++k) {
                            int64_t lev = (int64_t)ez * N + k;
                            for (int j = 0; j < P; ++j)
                                for (int i = 0; i < P; ++i) {
                                    int p[3];
                                    face_point(f, L, ex * N + i, ey * N + j, p);
                                    *g++ = (int32_t)(hid[p[0] + L1 * (p[1] + L1 * p[2])] + m.nh * lev);
                                }
                        }
                    }
    }
    if (d.kind == NUMA_MESH_SHELL) {
        // copies of each horizontal node in the bottom layer, ascending e*np + l
        // (the radial copies follow from the layer): the shell finish's lists
        const int64_t neh = 6 * (int64_t)d.ne[0] * d.ne[0], PP = (int64_t)P * P;
        m.hoff.assign(m.nh + 1, 0);
        for (int64_t eh = 0; eh < neh; ++eh)
            for (int64_t c = 0; c < PP; ++c) m.hoff[m.G[eh * np + c] + 1]++;
        for (int64_t h = 0; h < m.nh; ++h) m.hoff[h + 1] += m.hoff[h];
        m.hidx.resize(neh * PP);
        std::vector<int32_t> hc(m.hoff.begin(), m.hoff.end() - 1);
        for (int64_t eh = 0; eh < neh; ++eh)
            for (int64_t c = 0; c < PP; ++c) m.hidx[hc[m.G[eh * np + c]]++] = (int32_t)(eh * np + c);
    }
    // inverse map by counting sort: copies of each unique node in ascending e*np + l
    m.off.assign(m.nu + 1, 0);
    for (int64_t c = 0; c < m.nl; ++c) m.off[m.G[c] + 1]++;
    for (int64_t I = 0; I < m.nu; ++I) m.off[I + 1] += m.off[I];
    m.idx.resize(m.nl);
    std::vector<int32_t> cur(m.off.begin(), m.off.end() - 1);
    for (int64_t c = 0; c < m.nl; ++c) m.idx[cur[m.G[c]]++] = (int32_t)c;
    // unique ids in first-occurrence order of the element scan: grouped by the
    // element that first touches them, which is the order the stage finish
    // walks so that its gathers stay within a few adjacent element regions
    m.own.resize(m.nu);
    {
        std::vector<uint8_t> seen(m.nu, 0);
        int64_t n = 0;
        for (int64_t c = 0; c < m.nl; ++c) {
            const int32_t I = m.G[c];
            if (!seen[I]) {
                seen[I] = 1;
                m.own[n++] = I;
            }
        }
    }
    // the inverse map re-indexed in that order (copies of node own[t] at
    // tidx[toff[t] .. toff[t+1]), still ascending)
    m.toff.resize(m.nu + 1);
    m.tidx.resize(m.nl);
    m.toff[0] = 0;
    for (int64_t t = 0; t < m.nu; ++t) {
        const int32_t I = m.own[t];
        int32_t o = m.toff[t];
        for (int32_t c = m.off[I]; c < m.off[I + 1]; ++c) m.tidx[o++] = m.idx[c];
        m.toff[t + 1] = o;
    }
    return NUMA_OK;
}

static inline uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

uint64_t layout_workspace(Mesh &m, int32_t prec_mask, char *base)
{
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) {
        uint64_t at = o;
        o = align256(o + bytes);
        return base ? base + at : nullptr;
    };
    // lean: what the batched stages of the recomputed box metric read, and
    // the inverse map the geometry sums the recomputed mass over
    const bool lean = (prec_mask & NUMA_WS_LEAN) && m.d.kind == NUMA_MESH_BOX;
    DeviceView v;
    if (!lean) v.G = (int32_t *)take(4ull * m.nl);
    v.off = (int32_t *)take(4ull * (m.nu + 1));
    v.idx = (int32_t *)take(4ull * m.nl);
    if (m.d.kind == NUMA_MESH_SHELL) v.hlat = (int32_t *)take(12ull * m.nh);
    if (!lean) {
        v.met = (double *)take(80ull * m.nl);
        if (prec_mask & 2) v.met32 = (float *)take(40ull * m.nl);
    }
    v.ref = (double *)take(24ull * m.nu);
    v.M = (double *)take(8ull * m.nu);
    v.Minv = (double *)take(8ull * m.nu);
    v.MinvR = (double *)take(8ull * m.nu);
    if (m.d.kind == NUMA_MESH_SHELL) v.grav = (double *)take(24ull * m.nu);
    v.nrm = (double *)take(48ull * m.nh);
    v.xu = (double *)take(24ull * m.nu);
    if (m.d.kind == NUMA_MESH_BOX) v.hcol = (double *)take(32ull * m.d.ne[0] * m.d.ne[1] * m.P * m.P);
    if (m.d.kind == NUMA_MESH_SHELL) {
        const uint64_t ncol = 6ull * m.d.ne[0] * m.d.ne[0] * m.P * m.P;
        v.scol = (double *)take(8ull * 13 * ncol);
        v.slay = (double *)take(8ull * 4 * m.d.ne[2] * m.P);
        v.shid = (int32_t *)take(4ull * ncol);
        v.hoff = (int32_t *)take(4ull * (m.nh + 1));
        v.hidx = (int32_t *)take(4ull * ncol);
    }
    if (!lean) {
        v.own = (int32_t *)take(4ull * m.nu);
        v.toff = (int32_t *)take(4ull * (m.nu + 1));
        v.tidx = (int32_t *)take(4ull * m.nl);
        v.ev64 = (double *)take(40ull * m.nl);
        if (prec_mask & 2) v.ev32 = (float *)take(20ull * m.nl);
        v.qs = (double *)take(40ull * m.nu);
        v.qs2 = (double *)take(40ull * m.nu);
        if ((prec_mask & 4) && m.walls) v.imexLU = (double *)take(imex_factor_bytes(m));
    }
    v.D64 = (double *)take(8ull * kMaxP * kMaxP);
    v.D32 = (float *)take(4ull * kMaxP * kMaxP);
    v.xi64 = (double *)take(8ull * kMaxP);
    v.w64 = (double *)take(8ull * kMaxP);
    v.flag = (int32_t *)take(4);
    if (base) {
        m.dv = v;
        m.lean = lean;
    }
    return o;
}

}  // namespace numa
