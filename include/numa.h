/*
 * numa.h -- C ABI of the MI355X (gfx950) hot path of the NUMA spectral-element
 * dynamical core (Mueller et al., "Strong scaling for numerical weather
 * prediction at petascale with the atmospheric model NUMA", IJHPCA 2016).
 *
 * The path: the explicit right-hand side of the compressible Euler equations
 * in perturbation form (rho', u, v, w, theta') on hexahedral spectral elements
 * with Gauss-Lobatto-Legendre (GLL) quadrature of order N (Sec. "Spatial
 * Discretization", Eq. (discstrongform), Eq. (derivatives)); the direct
 * stiffness summation (DSS) weighted by the diagonal mass matrix; and an
 * explicit Runge-Kutta stage update (Sec. "Time Discretization"; Code example 1).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Status: every function returns int32_t: NUMA_OK (0) or a negative code.
 *   numa_last_error() returns a thread-local message for the last failure.
 *   Nothing aborts, throws or exits across this boundary.
 * - Device work is asynchronous on the caller's stream (a hipStream_t passed
 *   as void*; NULL is the default stream).  Device faults surface at the next
 *   synchronising call, as in HIP.  Argument errors are detected on the host
 *   before anything is enqueued.
 * - Memory: the library never allocates device memory.  The caller allocates
 *   one workspace of numa_mesh_workspace_bytes() and binds it with
 *   numa_mesh_attach_workspace(); states and outputs are caller-owned device
 *   buffers.  The mesh handle owns only host memory.
 * - Layouts: unique-node (CG storage) fields are structure-of-arrays
 *   [nvar][n_unique] FP64.  Element-local (E-vector, DG storage) fields are
 *   [nvar][n_elem][(N+1)^3] FP64 with local node l = i + (N+1)(j + (N+1)k).
 *   The state q is [5][n_unique]: rho', u, v, w, theta'.
 * - Threading: a handle is not thread-safe; distinct handles are independent.
 */
#ifndef NUMA_H
#define NUMA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NUMA_OK 0
#define NUMA_EINVAL -1      /* bad argument: null pointer, order, sizes, state of the handle */
#define NUMA_ENOMEM -2      /* workspace missing or too small */
#define NUMA_EDEVICE -3     /* a HIP runtime call failed */
#define NUMA_EUNSUPPORTED -4

#define NUMA_MESH_BOX 0     /* periodic in x and y; z periodic or bounded by no-flux walls */
#define NUMA_MESH_SHELL 1   /* equiangular cubed-sphere shell, no-flux bottom and top */

#define NUMA_PREC_FP64 0    /* everything in FP64 */
#define NUMA_PREC_MIXED 1   /* contractions, metric products and fluxes in FP32 */

#define NUMA_METRIC_STORED 0     /* metric terms and J w read per element-local node */
#define NUMA_METRIC_RECOMPUTE 1  /* box: recomputed in the element kernel every stage */

#define NUMA_STAGE_GATHER 0  /* element kernel writes J w R per copy; a finish kernel gathers the copies */
#define NUMA_STAGE_BLOCK 1   /* one kernel per block of element columns sums the copies in LDS */
#define NUMA_STAGE_COLOUR 2  /* 8 colour passes add J w R into a unique-node accumulator */
#define NUMA_STAGE_SPLIT 3   /* element kernel finishes its run's interior nodes; a face kernel the rest */
#define NUMA_STAGE_AUTO 4    /* default: NUMA_STAGE_SPLIT in FP64 where it applies, else NUMA_STAGE_GATHER */

#define NUMA_RK_SSP33 0      /* three-stage third-order SSP Runge-Kutta (Shu-Osher) */
#define NUMA_RK_SSP53 1      /* five-stage third-order SSP Runge-Kutta (Spiteri-Ruuth) */

#define NUMA_DSS_MASS 1     /* divide the summed contributions by the mass matrix */
#define NUMA_DSS_NOFLUX 2   /* project components 1..3 of a 5-variable field at walls */

/* numa_export selectors */
#define NUMA_FIELD_MASS 0        /* [n_unique] diagonal mass matrix M */
#define NUMA_FIELD_REF 1         /* [3][n_unique] rho_bar, theta_bar, p_bar */
#define NUMA_FIELD_COORDS 2      /* [3][n_unique] x, y, z of the unique nodes */
#define NUMA_FIELD_METRIC 3      /* [10][n_local] xi_x..zeta_z (row-major inverse Jacobian), J w */
#define NUMA_FIELD_GRAVITY 4     /* [3][n_unique] gravity vector */
#define NUMA_FIELD_LOCAL_COORDS 5 /* [3][n_local] element-local node coordinates */

typedef struct numa_mesh *numa_mesh_t;

/*
 * Mesh description.  order = N, the polynomial order p of the paper (N+1 GLL
 * points per direction), 1 <= N <= 8.
 * Box: ne = (nx, ny, nz) elements, periodic = (1, 1, 0 or 1), each periodic
 *   direction needs ne >= 2; extent = (Lx, Ly, H) in m; terrain_amp h0 gives
 *   the terrain-following map z' = z + h0 sin(2 pi x/Lx) sin(2 pi y/Ly)(1 - z/H).
 * Shell: ne = (ne, ignored, nz): ne x ne elements per cube face, nz radial
 *   layers; extent = (a, ignored, H): inner radius and depth.
 */
typedef struct numa_mesh_desc {
    int32_t kind;
    int32_t order;
    int32_t ne[3];
    int32_t periodic[3];
    double extent[3];
    double terrain_amp;
} numa_mesh_desc;

/* Gas and reference-atmosphere constants.  T0: theta0 of the isentropic box
 * reference, or the temperature of the isothermal shell reference. */
typedef struct numa_phys {
    double R, cp, g0, p0, T0;
} numa_phys;

/* Initial perturbation over the reference state (workload definition).
 * kind 0: rest; 1: cosine bubble theta' = amp (1 + cos(pi r/radius))/2 for
 * r < radius around c = (x, y, z); 2 (shell): zonal jet jet_u0 cos^2(lat) and a
 * gaussian theta' blob of e-folding lengths (radius, lz) at c = (lon, lat, height).
 * rho' = -rho_bar theta'/(theta_bar + theta') keeps the pressure unperturbed.
 * noise_amp scales the optional standard-normal noise added to u, v, w. */
typedef struct numa_ic {
    int32_t kind;
    double amp, radius;
    double c[3];
    double lz, jet_u0, noise_amp;
} numa_ic;

/* Thread-local description of the last error (never NULL). */
const char *numa_last_error(void);

/* GLL nodes xi[N+1], weights w[N+1], derivative matrix D[(N+1)^2] row-major,
 * D[i*(N+1)+m] = dpsi_m/dxi at xi_i (Sec. "Spatial Discretization").  Host only. */
int32_t numa_gll(int32_t order, double *xi, double *w, double *D);

/* Build the host mesh: numbering, element -> unique gather map and its inverse
 * (the paper's adjacency lookup table that enumerates the CG nodes, Sec. "Mesh
 * generation and load balancing").  Host only.  *out receives the handle. */
int32_t numa_mesh_create(const numa_mesh_desc *d, numa_mesh_t *out);
int32_t numa_mesh_destroy(numa_mesh_t m);

/* Sizes: elements, element-local nodes, unique nodes, unique nodes per level
 * (horizontal), levels.  Any pointer may be NULL. */
int32_t numa_mesh_info(numa_mesh_t m, int64_t *n_elem, int64_t *n_local, int64_t *n_unique,
                       int64_t *n_horiz, int64_t *n_levels);

/* Host copy of the gather map: host_out[e*(N+1)^3 + l] = unique id.  Host only. */
int32_t numa_mesh_gather_map(numa_mesh_t m, int32_t *host_out);

/* Device workspace needed for the precisions in prec_mask (bit 0: FP64 path,
 * bit 1: mixed path) and, with bit 2 (NUMA_WS_IMEX, meshes with walls), the factors
 * of numa_imex_step's vertical line systems (8 (4N+1) n_levels n_horiz bytes).
 * The FP64 data (geometry, reference, maps, scratch) is always included.
 * Bit 3 (NUMA_WS_LEAN; box meshes whose x element count fits the batched
 * finish) asks for only what batched steps with the recomputed metric read:
 * the reference state, M, M^-1, the recomputed metric's column factors and
 * mass, wall normals, coordinates and the inverse map; not the gather map,
 * the per-node metric, the first-occurrence copy lists, the contribution and
 * stage-state scratch nor the IMEX factors (at 64x64x16, N = 4: 0.36 GB
 * against 2.28 GB with both precisions).  On such a mesh numa_geometry forms
 * M as the sum of the recomputed J w (the same metric, to ~1e-14), and only
 * numa_geometry, numa_init_state, numa_export (not NUMA_FIELD_METRIC),
 * numa_rk_stage and the batched steps (numa_step_batch, its no-allocation
 * variant and captured graphs; recomputed metric, no filter) run on it:
 * the others return NUMA_ENOMEM. */
#define NUMA_WS_IMEX 4
#define NUMA_WS_LEAN 8
int32_t numa_mesh_workspace_bytes(numa_mesh_t m, int32_t prec_mask, uint64_t *bytes);

/* Bind a caller-owned device buffer (256-byte aligned) as the workspace.
 * The buffer must outlive every call on the handle.  NUMA_EUNSUPPORTED for
 * NUMA_WS_LEAN on a mesh the batched steps do not take. */
int32_t numa_mesh_attach_workspace(numa_mesh_t m, void *dev_ptr, uint64_t bytes, int32_t prec_mask);

/* Geometry (computed once, remark after Eq. (derivatives)): uploads the maps,
 * computes element-local coordinates, the metric terms and J w by derivative
 * contractions of the coordinates (isoparametric), the mass matrix
 * M_I = sum_e w_ijk J^e (Eq. (discstrongform)) and its inverse, the reference
 * state, gravity, wall normals, the column (and, shell, layer) factors of
 * the recomputed metric and the inverse of the mass summed from the
 * recomputed J w (used by the stages in NUMA_METRIC_RECOMPUTE mode), into
 * the workspace.  The hydrostatic reference state is computed here from ph
 * (not passed in): the box's isentropic profile with theta0 = ph->T0, or the
 * shell's isothermal one at T = ph->T0 with g = g0 (a/r)^2 (the paper's
 * equation set is cited, not stated: a reading), with p_bar re-evaluated from
 * the equation of state at every node; numa_export(NUMA_FIELD_REF) returns it.
 * Asynchronous.  NUMA_EINVAL for invalid constants (R, cp, p0, T0 > 0,
 * cp > R, g0 >= 0) or a box top at or above the isentropic model top;
 * NUMA_ENOMEM without a workspace. */
int32_t numa_geometry(numa_mesh_t m, const numa_phys *ph, void *stream);

/* Metric terms of the element kernels (numa_rhs, numa_step, numa_step_batch).
 * NUMA_METRIC_STORED (default) reads the 9 inverse-metric entries and J w
 * computed by numa_geometry at every element-local node.  NUMA_METRIC_RECOMPUTE
 * recomputes the same isoparametric metric in the kernel every stage from
 * factors that numa_geometry computes once, so the per-node metric costs no
 * memory traffic (the paper's next step, Sec. "Next Steps": recompute the
 * metric terms in each stage).  Box: four factors per element column and
 * local (i, j) of the terrain-following map (J w without w_k, 1/z_zeta and the
 * two terrain slopes over x_xi z_zeta, y_eta z_zeta).  Shell: per element
 * column and local (i, j) the three contravariant directions of the
 * equiangular map scaled by the triple product T, T w_i w_j and the radial
 * direction; per radial node 1/r, 1/h_zeta, r^2 h_zeta w_k and the gravity
 * g0 (a/r)^2 (the gather map and the gravity array are not read either).
 * Host only. */
int32_t numa_mesh_set_metric(numa_mesh_t m, int32_t mode);

/* How a fused stage of numa_step, numa_step_batch and numa_stage_rhs sums the
 * element contributions at the unique nodes (the DSS of the text after
 * Eq. (derivatives), inside the time loop of Code example 1).  Box meshes
 * with the recomputed metric; every mode gives the same sums up to their
 * order (parity with the oracle within 1e-12 either way), and every mode is
 * deterministic.
 * NUMA_STAGE_GATHER: the element kernel writes J w R of every
 *   element-local node (node-major), the finish kernel gathers the copies of
 *   each unique node in a fixed order; every mesh.
 * NUMA_STAGE_BLOCK: a workgroup owns a block of element columns and walks
 *   its element layers upwards, summing the copies in LDS and finishing the
 *   nodes whose copies all lie in the block; it recomputes the western
 *   neighbour element's east face itself, so x block faces are not shared,
 *   and writes partial sums only on its y faces (and its z faces between
 *   blocks), which a second kernel adds.  Meshes with walls, N = 2..4, nx a
 *   multiple of 4 (N = 4) or 8, ny even; the stage's input and output
 *   states must differ (numa_stage_rhs: r != q).
 * NUMA_STAGE_COLOUR: the elements are coloured by the parity of
 *   (ex, ey, ez); one launch per colour adds J w R with a plain read-modify-
 *   write into an FP64 accumulator [5][n_unique] in the workspace scratch (no
 *   two elements of a colour share a node: no atomics), the colours in a
 *   fixed order; a pointwise kernel then applies M^-1, the wall projection
 *   and the update (the paper's scheme of re-ordering elements so that
 *   concurrent threads never update the same node, Sec. "OpenMP").  N <= 4,
 *   nx, ny, nz even.
 * NUMA_STAGE_SPLIT: the element kernel's workgroup holds a run of
 *   consecutive elements along x; it adds the copies of the x faces shared
 *   inside the run in LDS and finishes every node whose copies it then holds
 *   (local j and k interior to the element, away from the x face that starts
 *   the run): M^-1, update, state.  The contributions of the other nodes
 *   (the element faces in y and z, and the run-start faces) go to the
 *   workspace scratch in rows along x, and a second kernel gathers them and
 *   finishes those nodes.  Recomputed metric; FP64 N = 1..8 (runs of
 *   64, 28, 16, 10, 7, 5, 4, 2 elements), mixed precision N <= 4; the stage
 *   may write its input state (the nodes the element kernel finishes are
 *   read by no other workgroup).
 * NUMA_STAGE_AUTO (default): NUMA_STAGE_SPLIT for FP64 stages where it
 *   applies, NUMA_STAGE_GATHER otherwise (the faster of the two in each
 *   precision on the 64 x 64 x 16 box, N = 3..8).
 * Meshes or stages a mode does not cover run NUMA_STAGE_GATHER.  NUMA_EINVAL
 * for an unknown mode.  Host only. */
int32_t numa_mesh_set_stage(numa_mesh_t m, int32_t mode);

/* Copy an internal field (NUMA_FIELD_*) to a caller device buffer. */
int32_t numa_export(numa_mesh_t m, int32_t what, void *dev_out, void *stream);

/* Initial state q [5][n_unique] (device) from ic; noise: device [3][n_unique]
 * standard normals or NULL.  Velocity is projected onto the walls. */
int32_t numa_init_state(numa_mesh_t m, const numa_ic *ic, const double *noise, double *q, void *stream);

/* Element-wise right-hand side (the paper's create_rhs): from the unique state
 * q [5][n_unique] to the element-local contributions c_elem [5][n_elem][(N+1)^3]
 * = J w_ijk R at every element-local node, with
 *   R_rho' = -div(rho u),  R_u = -(u.grad)u - grad(p')/rho + (rho'/rho) g,
 *   R_theta' = -u.grad(theta') [- u.grad(theta_bar) on the shell],
 * derivatives by Eq. (derivatives) (chain rule through the metric terms).
 * prec: NUMA_PREC_FP64 or NUMA_PREC_MIXED (requires a mixed workspace).
 * q and c_elem must not overlap. */
int32_t numa_rhs(numa_mesh_t m, int32_t prec, const double *q, double *c_elem, void *stream);

/* Direct stiffness summation (the text after Eq. (derivatives): the element
 * contributions are summed at the shared grid points and weighted by the
 * element volumes, i.e. divided by the diagonal mass M_I = sum_e w_ijk J^e of
 * Eq. (discstrongform); Code example 1: DSS and multiplication with the
 * inverse mass matrix) of an element-local field c_elem [nvar][n_local]
 * (device) into out [nvar][n_unique] (device): the sum over the copies of
 * each unique node, in ascending element-local order; NUMA_DSS_MASS divides
 * by M; NUMA_DSS_NOFLUX (nvar == 5) removes the wall-normal part of
 * components 1..3 (the no-flux walls, a reading: the paper states no
 * boundary condition).  c_elem and out must not overlap.  NUMA_EINVAL for a
 * null pointer, nvar < 1, unknown flags or NOFLUX with nvar != 5. */
int32_t numa_dss(numa_mesh_t m, int32_t nvar, const double *c_elem, double *out, int32_t flags,
                 void *stream);

/* Boyd-Vandeven filter (Sec. "Filter"; Code example 1: filter after the
 * stages, then DSS with the inverse mass matrix), in place on the state
 * q [5][n_unique] (device).  Each element's nodal values of every variable are
 * multiplied by F (x) F (x) F, F = V diag(sigma) V^-1 the 1D nodal filter
 * (V_ik = P_k(xi_i), Legendre polynomials at the GLL nodes), weighted by J w,
 * summed at the unique nodes, divided by M and projected at the walls: the
 * DSS of numa_dss with NUMA_DSS_MASS | NUMA_DSS_NOFLUX.  The paper names the
 * filter but not its parameters; here sigma_k = 1 for k <= cutoff and, with
 * t = (k - cutoff) / (N - cutoff), d = t - 1/2, the erfc-log form
 * sigma_k = erfc(2 sqrt(filter_order) d sqrt(-log(1 - 4 d^2) / (4 d^2))) / 2
 * (1/2 at t = 1/2, 0 for the top mode N); cutoff >= N leaves every element
 * unchanged.  filter_order must be finite and > 0, cutoff >= 0 (NUMA_EINVAL
 * otherwise).  The state is the perturbation state (rho', u, v, w, theta'), so
 * the hydrostatic reference is not filtered.  On a box whose FP64 stages
 * take the split DSS (numa_mesh_set_stage) the filter takes it too
 * (the same contributions, their copies summed in that schedule's order).  Uses the
 * mesh's contribution scratch, like numa_step: calls on one mesh on different
 * streams race. */
int32_t numa_filter(numa_mesh_t m, double filter_order, int32_t cutoff, double *q, void *stream);

/* The 1D filter matrix of numa_filter for GLL order `order` (1..8):
 * F[i * (order + 1) + m], host memory, (order + 1)^2 doubles.  Host only. */
int32_t numa_filter_matrix(int32_t order, double filter_order, int32_t cutoff, double *F);

/* One explicit Runge-Kutta stage update ("update q" of Code example 1;
 * Sec. "Time Discretization": the fully explicit scheme is a Runge-Kutta
 * method whose coefficients the text does not give; the reading used here is
 * SSP-RK3 in Shu-Osher form): stage s in 0..2, pointwise over [5][n_unique]
 * (device), qout = a_s qn + b_s (qs + dt r), (a, b) = (0, 1), (3/4, 1/4),
 * (1/3, 2/3); r is the DSS-ed right-hand side (numa_dss with
 * NUMA_DSS_MASS | NUMA_DSS_NOFLUX of numa_rhs).  qout may alias qs or qn; qn
 * is not read for s = 0.  NUMA_EINVAL for a null pointer or s outside 0..2. */
int32_t numa_rk_stage(numa_mesh_t m, int32_t stage, double dt, const double *qn, const double *qs,
                      const double *r, double *qout, void *stream);

/* The time loop of Code example 1 (per stage: create_rhs, DSS and the
 * multiplication with the inverse mass matrix, update q; Sec. "Time
 * Discretization"): nsteps Runge-Kutta steps in place on q [5][n_unique] (device) with the mesh's
 * integrator (numa_mesh_set_integrator; SSP-RK3 unless set), each stage being
 * rhs -> DSS (mass, no-flux) -> stage update, fused into two kernels: the
 * element kernel writes every element-local node's contribution J w R
 * (node-major: a copy's five values together); the finish kernel sums the
 * copies of each unique node, applies M^-1, the wall projection and the
 * update (the mesh's DSS schedule, numa_mesh_set_stage: by default in FP64
 * on the box the element kernel already sums the copies inside its run of
 * elements and finishes those nodes, and writes only the others' copies for
 * the finish kernel).  In FP64 (box and shell; not the generic box path, nor the box at
 * N = 5, 6 with the recomputed metric) the contribution
 * away from the walls is J w (q_s + c dt R), so that the finish need not read
 * q_s there; with the recomputed metric M is then the sum of the recomputed
 * J w.  Uses the workspace scratch; equals the composition of numa_rhs,
 * numa_dss and numa_rk_stage up to rounding of the state (the copies may be
 * summed in another order, and q_s enters through the weighted sum).
 * With a filter set on the mesh (numa_mesh_set_filter) every step ends with
 * numa_filter (Code example 1: the filter follows the stages).
 * The stream must not run other work on q or the workspace meanwhile.
 * The time loop as a HIP graph: the launches of one step are captured once
 * (on a stream of the mesh's own) and the graph is replayed nsteps times on
 * the caller's stream; the capture is kept for the next call while the
 * precision, dt, q and the mesh's settings (metric, stage mode, integrator,
 * filter, workspace, geometry) are unchanged, and redone otherwise.  Direct
 * launches instead while numa_profile is on, while the caller's stream is
 * itself being captured, or after numa_mesh_set_step_graph(m, 0).  Both give
 * bitwise the same result. */
int32_t numa_step(numa_mesh_t m, int32_t prec, double dt, int32_t nsteps, double *q, void *stream);

/* numa_step's captured step on (enable != 0, the default) or off (direct
 * launches; drops a kept capture).  Host only. */
int32_t numa_mesh_set_step_graph(numa_mesh_t m, int32_t enable);

/* The right-hand side of the time loop as numa_step's fused stage computes
 * it (Code example 1: create_rhs, then DSS and multiplication with the
 * inverse mass matrix; Eq. (discstrongform) with the DSS weights of the text
 * after Eq. (derivatives)): r [5][n_unique] (device, FP64) = M^-1 times the
 * sum over the copies of each unique node of J w R, with the wall-normal part
 * of components 1..3 removed at the no-flux walls.  It runs the same element
 * and finish kernels as numa_step (the kernel choice by order, metric mode and
 * precision; the copies summed in the same order; M^-1 of the same J w), as a
 * stage whose update is the identity on R, so no kernel folds a state into the
 * contributions.  Equals numa_dss(numa_rhs(q), NUMA_DSS_MASS | NUMA_DSS_NOFLUX)
 * up to rounding.  prec as for numa_rhs.  r must not alias q (NUMA_EINVAL:
 * the fused block stage finishes nodes while other workgroups still read q).  Uses the workspace
 * scratch like numa_step (calls on one mesh on different streams race). */
int32_t numa_stage_rhs(numa_mesh_t m, int32_t prec, const double *q, double *r, void *stream);

/* 1D-IMEX (Sec. "Time Discretization": implicit corrections along the vertical
 * columns after an explicit leap-frog step; Code example 1: IMEX corrections
 * per vertical column), nsteps steps on the pair (qprev = q^{n-1},
 * qcur = q^n), both [5][n_unique] on the device, updated in place to
 * (filtered q^n, q^{n+1}):
 *   q* = q^{n-1} + 2 dt L(q^n)   (a fused stage, L as in numa_step),
 *   (I - dt V) q^{n+1} = q* - dt V(2 q^n - q^{n-1})   (per vertical line),
 *   q^n <- q^n + ra (q^{n-1} - 2 q^n + q^{n+1})       (Robert-Asselin filter).
 * With n the unit vertical (z on the box, radial on the shell), w = u.n and
 * s = 1 (box) or r^2 (shell), V is the linearisation about the hydrostatic
 * reference of the vertical terms: V_rho' = -(1/s) d(s rho_bar w)/dn,
 * V_u = n (-(1/rho_bar) d p_L/dn + (g.n) rho'/rho_bar) with
 * p_L = (gamma p_bar/rho_bar)(rho' + rho_bar theta'/theta_bar),
 * V_theta' = -w d theta_bar/dn (zero on the isentropic box), discretised like
 * create_rhs (DSS, M^-1) with zero momentum rows at the walls; it acts along
 * each vertical lattice line (horizontal unique node h, levels h + n_h k) and
 * changes the velocity only along n.  The scheme's details are not in the
 * paper (it cites another); this is the reading used.  Meshes with no-flux
 * walls (the shell, and boxes not periodic in z; NUMA_EUNSUPPORTED otherwise,
 * and when a line of n_levels levels needs more than 64 KB of LDS); dt finite,
 * 0 <= ra < 1, distinct states (NUMA_EINVAL).  prec selects the explicit step's arithmetic; the line solves
 * are FP64.  The line matrices I - dt V depend only on dt and the reference
 * state: they are factored (band LU, in one workgroup per line) into the
 * workspace at the first call and whenever dt changes, so the workspace must
 * be attached with NUMA_WS_IMEX (NUMA_ENOMEM otherwise); each step then solves
 * all lines with one lane per line.  The mesh's filter and integrator settings
 * are not used.  Uses the workspace scratch like numa_step.  To start, pass
 * qprev = qcur (a forward first step) or a state one step back. */
int32_t numa_imex_step(numa_mesh_t m, int32_t prec, double dt, double ra, int32_t nsteps, double *qprev,
                       double *qcur, void *stream);

/* The time integrator of numa_step, numa_step_batch and numa_batch_capture
 * (Sec. "Time Discretization": explicit Runge-Kutta; the paper's scheme has
 * five stages and third order, its coefficients are not in the text):
 * NUMA_RK_SSP33, the three-stage third-order SSP scheme in Shu-Osher form
 * (default), or NUMA_RK_SSP53, the optimal five-stage third-order SSP scheme
 * of Spiteri and Ruuth (SIAM J. Numer. Anal. 40(2), 2002):
 *   u1 = u0 + b10 dt L(u0), u2 = u1 + b21 dt L(u1),
 *   u3 = a30 u0 + a32 u2 + b32 dt L(u2), u4 = a40 u0 + a43 u3 + b43 dt L(u3),
 *   q^{n+1} = a52 u2 + a54 u4 + b54 dt L(u4)
 * (15-digit coefficients in api.cpp).  Every stage is one fused stage as in
 * numa_step; SSP53 keeps a second stage state (in the workspace, and in batch
 * scratch: numa_step_scratch_bytes grows by 40 n_unique bytes, so size the
 * scratch after choosing the integrator).  NUMA_EINVAL for an unknown value.
 * Host only. */
int32_t numa_mesh_set_integrator(numa_mesh_t m, int32_t integrator);

/* Make numa_step, numa_step_batch and numa_batch_capture end every step with
 * numa_filter(m, filter_order, cutoff) on the state (enable != 0), or stop
 * doing so (enable == 0: the other arguments are ignored).  Parameters as for
 * numa_filter (NUMA_EINVAL otherwise).  The filter of a batch item uses its
 * mesh's scratch, one item after another on the batch's stream, so items may
 * share a mesh; a captured graph keeps the setting of its capture.  Host
 * only. */
int32_t numa_mesh_set_filter(numa_mesh_t m, int32_t enable, double filter_order, int32_t cutoff);

/* ---- Batched stages (continuous batching of independent solves) ----
 * An item is one solve: a mesh whose geometry may be shared with other items
 * (read only), its state q [5][n_unique] (device, updated in place), private
 * device scratch of at least numa_step_scratch_bytes() (256-byte aligned; its
 * size in scratch_bytes, NUMA_ENOMEM if short), and its dt.
 * numa_step_batch advances all items by nsteps Runge-Kutta steps with one
 * element launch and one finish launch per stage for every 16 items.  All
 * items must have the same order, precision, metric mode and integrator, be
 * box meshes whose x element
 * count is a multiple of the finish segment (4 for N <= 6, 2 for N = 7, 8),
 * and have distinct states and scratch.  Each item's result is bitwise the
 * result of numa_step on it alone (the same per-element and per-node code),
 * the filter of its mesh included. */
typedef struct numa_batch_item {
    numa_mesh_t mesh;
    double *q;
    void *scratch;
    uint64_t scratch_bytes;  /* size of scratch: at least numa_step_scratch_bytes() */
    double dt;
    int32_t *nonfinite;      /* device, or NULL: set to 1 (never cleared) when a stage
                                writes a non-finite value into the item's state */
} numa_batch_item;

int32_t numa_step_scratch_bytes(numa_mesh_t m, int32_t prec, uint64_t *bytes);
int32_t numa_step_batch(const numa_batch_item *items, int32_t n, int32_t prec, int32_t nsteps, void *stream);

/* ---- Batched steps without device allocation ----
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * numa_step_batch with each item's scratch taken from a static device array
 * of the library, NUMA_NOALLOC_SCRATCH_BYTES on each GPU it runs on (held
 * from the first call there until the process ends), instead of a caller
 * buffer.  Items, precision, step count and results are as numa_step_batch's
 * (the same kernels: bitwise the same results), except that every item's
 * scratch must be NULL and its scratch_bytes 0.  The items' scratch lies one
 * after another in the array, numa_step_scratch_bytes() each: NUMA_ENOMEM
 * when the sum exceeds NUMA_NOALLOC_SCRATCH_BYTES; NUMA_EINVAL for more than
 * NUMA_NOALLOC_MAX_ITEMS items or a mesh that is profiling.  No device or
 * host allocation.  Runs on the current device; the first call on a device
 * looks up the array's address there, and a call with nsteps = 0 does only
 * that (items are not read): make one before capturing the call into a graph.
 * Nothing in the array needs to start at zero (every stage writes its
 * scratch before reading it).  All calls on one GPU share its array, which
 * keeps the last call's contents: calls that overlap in time on one GPU
 * (other streams, host threads, or graph replays) race and give wrong
 * results.  The meshes' workspaces (geometry, the filter's scratch) remain
 * the caller's, attached beforehand. */
#define NUMA_NOALLOC_SCRATCH_BYTES (128ull << 20)
#define NUMA_NOALLOC_MAX_ITEMS 64
int32_t numa_step_batch_noalloc(const numa_batch_item *items, int32_t n, int32_t prec, int32_t nsteps, void *stream);

/* Capture numa_step_batch(items, n, prec, nsteps) on a non-default stream into
 * a HIP graph (no memory operations inside); numa_graph_launch replays it on
 * any stream with the same arguments (the same device buffers), so membership
 * changes need a new capture.  The items' meshes must not be profiling. */
typedef struct numa_graph *numa_graph_t;
int32_t numa_batch_capture(const numa_batch_item *items, int32_t n, int32_t prec, int32_t nsteps, void *stream,
                           numa_graph_t *out);
int32_t numa_graph_launch(numa_graph_t g, void *stream);
int32_t numa_graph_destroy(numa_graph_t g);

/* Per-kernel timing of numa_step: while enabled, numa_step records HIP events
 * on the caller's stream around each launch of its two stage kernels (the
 * element kernel and the DSS/update finish).  numa_profile(m, 1) starts a new
 * accumulation, numa_profile(m, 0) stops recording.  numa_profile_read waits
 * for the recorded events and writes out[0] = total element-kernel ms,
 * out[1] = its launches, out[2] = total finish ms, out[3] = its launches. */
int32_t numa_profile(numa_mesh_t m, int32_t enable);
int32_t numa_profile_read(numa_mesh_t m, double *out);

#ifdef __cplusplus
}
#endif
#endif /* NUMA_H */
