/*
 * fnpf.h - C ABI of the MI355X (gfx950) FNPF-SEM per-stage Laplace-solve library.
 *
 * The library implements, on one GPU, the hot path of the fully nonlinear
 * potential-flow spectral element model of Visbech, Melander and
 * Engsig-Karup ("FNPF-SEM", 2025): at every explicit RK4 stage
 *   Step 4.1  move the extruded mesh to the current surface elevation eta,
 *   Step 4.2  impose phi = phi_eta on the free surface (Dirichlet),
 *   Step 4.3  solve the Laplace problem (Eq. 1, weak form Eq. 4) by PCG,
 *   Step 4.4-4.5  recover the vertical velocity w_eta at the surface,
 *   Step 4.6  evaluate the Zakharov free-surface conditions (Eqs. 2-3),
 *   Step 3    accumulate the ERK4 stages (Sec. 3.2),
 *   Step 4.7  apply relaxation zones (Sec. 3.3).
 *
 * Discretisation (readings of the paper where it is silent):
 *   - hexahedral elements extruded from quadrilaterals (3D) or intervals
 *     (2D x-z slices); GLL nodes of degree p with collocated GLL quadrature;
 *   - node level v of a column sits at z = -h + sigma_v (eta + h);
 *   - volume vectors are layer-major: index = v * n_s + hn, v = 0 (bottom)
 *     .. p*nz (free surface), hn the horizontal node; the paper's surface
 *     map m is therefore the slice [p*nz*n_s, (p*nz+1)*n_s);
 *   - w recovery is the lumped-GLL L2 projection of d(phi)/dz; the
 *     free-surface right-hand side uses the lumped GLL surface mass.
 *
 * Conventions for every entry point:
 *   - Array arguments documented as "device" are device pointers on the
 *     context's GPU, owned by the caller, contiguous, 8-byte (double) or
 *     4-byte (float) elements.  "host" arrays are read (or written) during
 *     the call only.  The library never keeps a caller pointer after a call
 *     returns; it owns only its internal workspaces, freed by fnpf_destroy.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream).
 *     Calls that need a scalar answer (fnpf_solve, fnpf_rk4_step and the
 *     adjoint solve) synchronise the stream; all others are asynchronous.
 *   - Every call returns a status and never aborts or throws across the ABI.
 *     Argument validation happens before any HIP call.  fnpf_last_error
 *     returns a message for the last failing call on a context.
 *   - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef FNPF_H
#define FNPF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fnpf_ctx_s *fnpf_ctx;

typedef enum {
  FNPF_OK = 0,
  FNPF_ERR_ARG = 1,       /* invalid argument (null pointer, size, ordering of calls) */
  FNPF_ERR_ALLOC = 2,     /* device or host allocation failed */
  FNPF_ERR_HIP = 3,       /* a HIP runtime call failed */
  FNPF_ERR_GEOM = 4,      /* eta + h <= 0 at some node, or a non-positive Jacobian */
  FNPF_ERR_NOCONV = 5,    /* PCG reached max_iter before rtol/atol */
  FNPF_ERR_BREAKDOWN = 6, /* p^T A p <= 0 in PCG */
  FNPF_ERR_NAN = 7,       /* NaN/Inf in the residual */
  FNPF_ERR_STATE = 8      /* call sequence error, e.g. an apply before any fnpf_geom */
} fnpf_status;

typedef enum { FNPF_F64 = 0, FNPF_F32 = 1 } fnpf_dtype;

/* Mesh description (host data, copied by fnpf_create).
 * dim 2: vertical x-z slice, horizontal elements are intervals;
 * dim 3: horizontal elements are quadrilaterals.  nh = (p+1)^(dim-1).
 *   eh_nodes    [n_eh][nh]   global horizontal node id (0..n_s-1) of each
 *                            element-local GLL node, local order i (xi)
 *                            fastest then j (eta); periodicity is folded in.
 *   eh_corner   [n_eh][2^(dim-1)][dim-1]  unwrapped physical corners; quads
 *                            ordered (-1,-1),(+1,-1),(+1,+1),(-1,+1) and
 *                            counter-clockwise; intervals (-1),(+1).
 *   eh_arc      NULL or [n_eh][4][3]: per quad edge (cx, cy, R) of a circle
 *                            the edge follows (R = 0 straight).  Edges:
 *                            e0 c0->c1, e1 c1->c2, e2 c3->c2, e3 c0->c3,
 *                            parametrised linearly in angle (shorter arc).
 *                            Interior node positions follow the Gordon-Hall
 *                            transfinite map of the four edges.
 *   eh_face_tag NULL or [n_eh][2(dim-1)]: 0 interior/periodic, 1 wall,
 *                            2 body (both impermeable: natural Neumann).
 *                            Quad sides are ordered like the edges; interval
 *                            sides are (xi=-1, xi=+1).
 *   layer_s     NULL (uniform) or [nz+1] increasing fractions, 0 .. 1.
 *   g           gravitational acceleration.                                */
typedef struct {
  int32_t dim;
  int32_t p;          /* 1 .. 8 */
  int32_t nz;         /* >= 1 */
  int32_t n_eh;       /* >= 1 */
  int64_t n_s;
  const int32_t *eh_nodes;
  const double *eh_corner;
  const double *eh_arc;
  const int32_t *eh_face_tag;
  const double *layer_s;
  double g;
} fnpf_mesh_desc;

/* PCG options.
 *   precision 0: FP64 PCG.  1: mixed - FP64 outer defect correction
 *                (residual with the FP64 operator, FP64 solution update)
 *                around an FP32 inner PCG (FP32 geometric factors, vectors
 *                and apply; FP64 dot products and scalars).
 *   precond   0: none (CG on A_II).  1: Jacobi (assembled diagonal).
 *             2: p-multigrid V-cycle (the paper's CG uses algebraic
 *                multigrid, Sec. 4): levels of degree p, p/2, ..., 1 on the
 *                same mesh, each a context of this library with its geometry
 *                interpolated from eta + h and h; tensor-product Lagrange
 *                interpolation between levels and its transpose; Chebyshev
 *                smoothing of D^-1 A of degree cheb_degree before and after
 *                each coarse correction (interval [lmax/24, lmax], lmax 1.1x an
 *                estimate of the largest eigenvalue of D^-1 A: 20 Lanczos
 *                steps on first use, then one power iteration from the Ritz
 *                vector after every fnpf_geom)
 *                and 10 Chebyshev steps on the degree-1 level.  The V-cycle is
 *                a fixed SPD operator, so the outer iteration is plain CG.
 *                The levels are built on first use (device memory about 0.3x
 *                of the fine level's vectors per precision).
 *   Stop when ||r||_2 <= max(rtol ||b||_2, atol), b = f_I - A_IS phi_s
 *   (unpreconditioned 2-norms over the non-surface nodes).
 *   max_iter bounds the total PCG iterations (inner ones for mixed);
 *   check_every is the number of iterations between host convergence checks
 *   (the iterations after convergence are skipped on the device, so results
 *   do not depend on it).  inner_rtol: relative reduction of each inner FP32
 *   solve, which also stops as soon as its residual is below half the outer
 *   tolerance; max_outer bounds the defect-correction sweeps.
 *   extrapolate (fnpf_rk4_step and fnpf_rk4_step_vjp): k = 1..4
 *   extrapolates the initial guess of stage s of a step in time from the
 *   same stage of the previous k + 1 steps taken with the same dt, with the
 *   polynomial of degree k through them: phi(n) = sum_{j=1}^{k+1}
 *   (-1)^(j+1) binom(k+1, j) phi(n-j) (k = 1: 2 phi(n-1) - phi(n-2));
 *   lower degrees while fewer steps exist.  It keeps k + 1 potentials [n_v]
 *   per stage on the device (a change of k starts a new history).  0 starts
 *   every stage from the previous stage's potential.  Only the initial
 *   guess changes; the converged solution meets the same tolerance.         */
typedef struct {
  int32_t precision;
  int32_t precond;
  double rtol;
  double atol;
  int32_t max_iter;
  int32_t check_every;
  double inner_rtol;
  int32_t max_outer;
  int32_t extrapolate;
  int32_t cheb_degree;   /* precond 2: smoothing degree, 1 .. 8 (default 2) */
  int32_t use_graph;     /* 1: the check_every iterations between host checks are captured
                            once as a HIP graph and replayed (default); 0: launched one by one.
                            Results are identical. */
  int32_t line_smoother; /* precond 2: 0 (default) Chebyshev smoothing of D^-1 A (point
                            Jacobi); 1 of B^-1 A, B the vertical line blocks of A_II (the
                            unknowns of one vertical node line coupled, banded with half
                            bandwidth p), factored by Cholesky after every geometry update, for
                            meshes whose thin layers couple the vertical strongly; every level
                            uses it and the smoothing intervals come from Lanczos / power
                            iterations in the B inner product. */
} fnpf_solve_opts;

typedef struct {
  int32_t iters;        /* PCG iterations (inner iterations summed for mixed) */
  int32_t outer_iters;  /* FP64 residual evaluations of the mixed path (0 for FP64) */
  double rel_res;       /* final FP64 ||r|| / ||b|| */
  double bnorm;         /* ||b||_2 */
} fnpf_solve_info;

/* Defaults: FP64, p-multigrid (precond 2), rtol 1e-8, atol 0, max_iter 20000,
 * check_every 8, inner_rtol 1e-6, max_outer 30, extrapolate 4, cheb_degree 2, use_graph 1,
 * line_smoother 0. */
void fnpf_default_opts(fnpf_solve_opts *opts);

/* Create a context on the current HIP device: validates and copies the mesh,
 * computes GLL data, horizontal metrics (Gordon-Hall coordinates), the greedy
 * column colouring used for conflict-free scatter, and allocates the FP64
 * workspaces (FP32 ones on first mixed use).  Errors: ARG (invalid mesh, e.g.
 * node ids out of range or unused, a non-positive horizontal Jacobian), ALLOC,
 * HIP.  *out is NULL on failure. */
fnpf_status fnpf_create(const fnpf_mesh_desc *mesh, fnpf_ctx *out);
fnpf_status fnpf_destroy(fnpf_ctx ctx);
/* Message of the last failing call on ctx; with ctx == NULL, the message of
 * the last failed fnpf_create on this thread. */
const char *fnpf_last_error(fnpf_ctx ctx);
const char *fnpf_status_string(fnpf_status s);

/* Sizes: volume nodes n_v = n_s (p nz + 1), surface nodes n_s, elements
 * n_e = n_eh nz, number of colours of the column colouring. Any pointer may be NULL. */
fnpf_status fnpf_sizes(fnpf_ctx ctx, int64_t *n_v, int64_t *n_s, int64_t *n_e, int32_t *n_colours);

/* GLL data of degree p (host, no context): nodes[p+1], weights[p+1] and
 * D[(p+1)*(p+1)] row-major, D[i*(p+1)+j] = l_j'(x_i).  Any output may be NULL. */
fnpf_status fnpf_gll(int32_t p, double *nodes, double *weights, double *D);

/* Host copy of the physical coordinates of every horizontal node:
 * xy[n_s][dim-1] (periodic nodes: the first element's image). */
fnpf_status fnpf_node_coords(fnpf_ctx ctx, double *xy);

/* Surface interpolation weights, for observation operators such as the wave gauges at which
 * the paper compares surface elevations (Sec. 4.2).  For each of n_pts points pts[n_pts][dim-1]
 * (host, physical horizontal coordinates, periodic directions unwrapped as in eh_corner), the
 * horizontal element containing it (the first in element order whose isoparametric map, the
 * degree-p interpolant of its GLL node positions, has a Newton inverse in [-1, 1]^(dim-1)) and
 * the degree-p Lagrange weights of that element's nh nodes: f(pt) = sum_t w[k][t]
 * f[node[k][t]] for a surface field f[n_s].  node[n_pts][nh] and w[n_pts][nh] are host arrays
 * written by the call.  Errors: ARG for a point outside the mesh, n_pts < 0 or NULL arrays. */
fnpf_status fnpf_surface_interp_weights(fnpf_ctx ctx, int32_t n_pts, const double *pts, int32_t *node, double *w);

/* Stiffness-apply variant (all compute the same operator, paper Eq. 4):
 *   0 (default) fused geometry: the per-point factors are re-evaluated in
 *     registers from five numbers per column node (eta+h, h and their
 *     horizontal derivatives) and the static horizontal metrics, so an apply
 *     reads x and writes y only.  3D: line schedule (below) with
 *     owner-computes assembly -- one launch over all columns, in which the
 *     columns of a workgroup (256 / (p+1)^2 consecutive ones) form a tile
 *     that sums its shared nodes in LDS and stores the nodes it owns (a node
 *     belongs to the tile of the lowest-numbered column that has it) and its
 *     other sums into face slots; a second launch adds the slots to the
 *     owners.  It is fastest
 *     when each column's own nodes are numbered consecutively (shared ones
 *     first); any consistent numbering gives the same result.  The
 *     kernels index with 32-bit byte offsets: when n_v * 8 bytes or the
 *     face slots, (p*nz+1) * n_slots * 8 bytes, reach 4 GiB (n_v >= 2^29,
 *     about 537 million nodes) the apply falls back to the colour assembly
 *     of 6 while n_v * sizeof(element) stays below 4 GiB, else to that of
 *     7; the result is the same.  2D: colour schedule with read-add-write
 *     of shared nodes;
 *   1 stored factors: fnpf_geom stores G (6 or 3 per point, FP64 and FP32)
 *     and the apply streams it from HBM;
 *   6 fused geometry, line schedule with colour assembly (3D): in the
 *     horizontal contraction phases each thread owns one xi-line and one
 *     eta-line of the element, so derivative coefficients are uniform
 *     scalars (2D: same as 7);
 *   7 fused geometry, colour schedule (one thread per vertical node line,
 *     derivatives through LDS reads).
 * Switching to 1 invalidates the current geometry (call fnpf_geom again).
 * Errors: ARG for any other value. */
fnpf_status fnpf_set_apply_variant(fnpf_ctx ctx, int32_t variant);

/* Enable the FP32 path: allocates FP32 factors and the inner-PCG vectors;
 * every later fnpf_geom also produces the FP32 factors.  fnpf_rk4_step with
 * precision 1 enables it by itself. */
fnpf_status fnpf_enable_fp32(fnpf_ctx ctx);

/* Step 4.1: per-point geometric factors for surface elevation eta[n_s] and
 * depth h[n_s] (device, FP64): G = w_q det(J) J^{-1} J^{-T} (6 symmetric
 * entries in 3D, 3 in 2D), the assembled Jacobi diagonal of the Laplace
 * operator, and FP32 copies when the mixed path is in use.  A node with
 * eta + h <= 0 raises a device flag reported as FNPF_ERR_GEOM by the next
 * synchronising call (fnpf_solve, fnpf_rk4_step, fnpf_sync). */
fnpf_status fnpf_geom(fnpf_ctx ctx, const double *eta, const double *h, void *stream);

/* Device copies of the factors of the last fnpf_geom (parity checks):
 * G[n_e][ng][(p+1)^dim] (ng = 6 in 3D ordered 00,01,02,11,12,22; 3 in 2D
 * ordered 00,01,11; element e = column * nz + layer; local node (k, j, i),
 * i fastest) in FP64 (dtype F64) or FP32, and diag[n_v] FP64.  Either may be NULL. */
fnpf_status fnpf_export_geometry(fnpf_ctx ctx, fnpf_dtype dtype, void *G, double *diag, void *stream);

/* Eq. 4: y = A x with the matrix-free sum-factorised stiffness operator of
 * the current geometry, x and y [n_v] device arrays of `dtype` (F32 uses the
 * FP32 factors).  mask_dirichlet != 0 sets the free-surface rows of y to 0.
 * x and y must not overlap.  Errors: STATE if fnpf_geom was never called
 * (or, for F32, never called since the FP32 path was enabled). */
fnpf_status fnpf_laplace_apply(fnpf_ctx ctx, fnpf_dtype dtype, const void *x, void *y, int32_t mask_dirichlet,
                               void *stream);

/* Allocation-free variant of fnpf_laplace_apply, for callers that cannot allocate device memory
 * during the call: code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, operator and result as fnpf_laplace_apply (bitwise identical).
 * The owner-computes schedule's face slots, which fnpf_laplace_apply keeps in the context,
 * live here in one library-wide device array of 128 MiB per GPU (allocated when the library's
 * device code is loaded, held until the process ends); the call allocates nothing.  Every call
 * on a GPU uses that GPU's one array: calls that overlap on a GPU (other streams, other
 * contexts, other host threads) race and must be serialised by the caller.  The slots are
 * written before they are read within each call, so nothing carries over between calls.
 * Errors: ARG when the face slots, (p nz + 1) * n_tile_slots elements of the dtype, exceed the
 * array (then use fnpf_laplace_apply); as fnpf_laplace_apply otherwise. */
fnpf_status fnpf_laplace_apply_noalloc(fnpf_ctx ctx, fnpf_dtype dtype, const void *x, void *y,
                                       int32_t mask_dirichlet, void *stream);

/* The vertical line smoother's block solve (opts.line_smoother): z = B^-1 r on the unknowns and
 * z = 0 on the free-surface level, B the vertical line blocks of A_II for the current geometry
 * (for horizontal node n, the principal submatrix of the Laplace operator on levels
 * 0 .. p nz - 1 of its node line), through their Cholesky factors, which this call (re)builds.
 * The smoother stands in for the multigrid the paper's Laplace solves use (Sec. 4, solver
 * settings).  r, z [n_v] device arrays of dtype (F32: factors rounded from FP64); no aliasing.
 * Errors: STATE before fnpf_geom (F32: without FP32 data); GEOM if a block is not positive
 * definite. */
fnpf_status fnpf_line_smoother_apply(fnpf_ctx ctx, fnpf_dtype dtype, const void *r, void *z, void *stream);

/* Eq. 1 boundary data: f_i = sum over the bottom and the wall/body faces of
 * int (q . n) l_i dS for a nodal flux field q[dim][n_v] (device, FP64,
 * physical components x, (y,) z), with the current geometry.  f[n_v] device. */
fnpf_status fnpf_neumann_load(fnpf_ctx ctx, const double *q, double *f, void *stream);

/* Steps 4.2-4.3: solve the Laplace problem with phi = phi_surface[n_s] on the
 * free surface and Neumann load neumann_f[n_v] (NULL = homogeneous).  phi[n_v]
 * (device) holds the initial guess on entry (its surface level is
 * overwritten) and the solution on exit; on NOCONV/BREAKDOWN it holds the last
 * iterate.  info (host, may be NULL) is filled in every case. */
fnpf_status fnpf_solve(fnpf_ctx ctx, const double *phi_surface, const double *neumann_f, double *phi,
                       const fnpf_solve_opts *opts, fnpf_solve_info *info, void *stream);

/* Steps 4.4-4.5: w_s[n_s] = recovered d(phi)/dz at the free-surface nodes for
 * phi[n_v] and the geometry of the last fnpf_geom (eta, h of that call). */
fnpf_status fnpf_w_surface(fnpf_ctx ctx, const double *phi, double *w_s, void *stream);

/* Step 4.6 / Eqs. 2-3: deta[n_s], dphi[n_s] from eta, phi_s, w_s [n_s] (all device FP64). */
fnpf_status fnpf_rhs(fnpf_ctx ctx, const double *eta, const double *phi_s, const double *w_s, double *deta,
                     double *dphi, void *stream);

/* Step 4.7 relaxation zones (host arrays [n_s], copied): after every full
 * step f <- (1 - cr) f + cr * ramp(t) * (f_c cos(omega t) + f_s sin(omega t))
 * for f = eta (eta_c, eta_s) and phi_s (phi_c, phi_s_); ramp(t) =
 * (1 - cos(pi t / t_ramp))/2 for t < t_ramp, else 1 (t_ramp <= 0: 1).
 * cr == NULL removes the relaxation. */
fnpf_status fnpf_set_relaxation(fnpf_ctx ctx, const double *cr, const double *eta_c, const double *eta_s,
                                const double *phi_c, const double *phi_s_, double omega, double t_ramp);

/* Free-surface form (Eq. 5; over-integration, Sec. 3.2).  nq = 0 (default):
 * collocated GLL quadrature with the lumped surface mass, so the RHS is
 * pointwise.  p + 1 <= nq <= 24: the consistent form; the integrands of
 * Eqs. 2-3 are evaluated at nq Gauss-Legendre points per direction of each
 * surface element and tested against the Lagrange basis, and the consistent
 * surface mass system is solved for d eta/dt and d phi_s/dt by a fixed-length
 * Chebyshev iteration preconditioned with the lumped mass (its interval is
 * bounded from the element Jacobians; the length gives a 1e-15 contraction).
 * nq >= (5p - 1)/2 integrates every term exactly on affine elements.  Used by
 * fnpf_rhs, fnpf_rhs_vjp, fnpf_rk4_step and fnpf_rk4_step_vjp; ignored in
 * linear mode, whose integrands lie in the discrete space (both forms agree).
 * Synchronises the device.  Errors: ARG for nq out of range, GEOM for a
 * non-positive Jacobian at a Gauss point. */
fnpf_status fnpf_set_surface_quadrature(fnpf_ctx ctx, int32_t nq);

/* Current nq, Chebyshev iteration count and eigenvalue interval of the
 * consistent surface solve (any pointer may be NULL). */
fnpf_status fnpf_surface_quadrature_info(fnpf_ctx ctx, int32_t *nq, int32_t *iters, double *lam_lo,
                                         double *lam_hi);

/* p-multigrid diagnostics (precond 2): *levels = number of levels (this one
 * and its coarse levels; 0 before the first multigrid solve builds them) and,
 * for the first min(levels, cap) levels from the finest, the current estimate
 * of the largest eigenvalue of D^-1 A on the unknowns that sets the Chebyshev
 * intervals (the value before the 1.1 safety factor; 0 where that precision
 * has not been refreshed yet).  lam64, lam32: host arrays of cap entries, or
 * NULL; reading them synchronises the device.  Errors: ARG for cap < 0. */
fnpf_status fnpf_multigrid_info(fnpf_ctx ctx, int32_t *levels, double *lam64, double *lam32, int32_t cap);

/* Modal filter of surface fields (Sec. 3.2, modal filtering; the paper's
 * triangles become tensor-product quads/intervals here).  Per surface
 * element, nodal values -> modal coefficients in the orthonormal Legendre
 * product basis (inverse Vandermonde at the GLL nodes) -> mode (n, m) scaled
 * by sigma(n) sigma(m) -> nodal values; a node shared by several elements
 * takes the mean of their results.  sigma(n) = 1 for n <= cutoff, else
 * exp(-alpha ((n - cutoff)/(p - cutoff))^order).
 * fnpf_set_modal_filter sets the filter (0 <= cutoff < p, alpha >= 0,
 * order >= 1); cutoff < 0 removes it.  While set, fnpf_rk4_step filters eta
 * and phi_s after every step (after relaxation) and fnpf_rk4_step_vjp applies
 * the transpose first.  Errors: ARG for parameters out of range. */
fnpf_status fnpf_set_modal_filter(fnpf_ctx ctx, int32_t cutoff, double alpha, int32_t order);

/* out[n_s] = filtered f[n_s] (device FP64, out must not alias f).
 * Errors: STATE if no filter is set. */
fnpf_status fnpf_modal_filter(fnpf_ctx ctx, const double *f, double *out, void *stream);

/* VJP of fnpf_modal_filter: f_bar (+=) [n_s] from out_bar [n_s] (no aliasing). */
fnpf_status fnpf_modal_filter_vjp(fnpf_ctx ctx, const double *out_bar, double *f_bar, void *stream);

/* Linear potential flow (the linearised model of Sec. 2.1, small-amplitude
 * limit of Eqs. 2-3): linear != 0 makes fnpf_rk4_step, fnpf_rk4_step_vjp,
 * fnpf_rhs and fnpf_rhs_vjp use the fixed domain at eta = 0 (the Laplace
 * problem is solved in -h <= z <= 0 with phi = phi_s on z = 0) and the linear
 * free-surface conditions d eta/dt = w, d phi_s/dt = -g eta.  The default
 * (0) is the fully nonlinear model.  fnpf_geom, fnpf_solve and fnpf_w_surface
 * are unaffected (they take the geometry they are given).  The flat geometry
 * is computed by the first linear step for a depth array and kept while the
 * same h pointer is passed and no other call replaces the geometry; after
 * changing h in place, call fnpf_set_linear(ctx, 1) again. */
fnpf_status fnpf_set_linear(fnpf_ctx ctx, int32_t linear);

/* One ERK4 step (Sec. 3.2) of the Zakharov system from time t with step dt,
 * in place on eta[n_s] and phi_s[n_s] (device FP64), depth h[n_s] (device),
 * followed by relaxation at t + dt.  The volume potential of the previous
 * stage is the PCG warm start (kept in the context).  tape (device, may be
 * NULL) receives, per stage s = 0..3, a record of n_v + 2 n_s doubles:
 * the stage's volume potential, then its surface elevation and surface
 * potential (tape[s*(n_v+2 n_s) ...]); it is the input of fnpf_rk4_step_vjp.
 * info (host, may be NULL) receives one record per stage. */
fnpf_status fnpf_rk4_step(fnpf_ctx ctx, double *eta, double *phi_s, const double *h, double t, double dt,
                          const fnpf_solve_opts *opts, double *tape, fnpf_solve_info *info, void *stream);

/* ---- Adjoint (vector-Jacobian products).  The paper has no adjoint; these
 * differentiate the discrete path above exactly (up to the solver tolerance).
 * "(+=)" marks device arrays that are accumulated into, never overwritten. */

/* VJP of fnpf_rhs: given deta_bar, dphi_bar [n_s], adds the contributions to
 * eta_bar (+=), phis_bar (+=) and w_bar (+=) [n_s]. */
fnpf_status fnpf_rhs_vjp(fnpf_ctx ctx, const double *eta, const double *phi_s, const double *w_s,
                         const double *deta_bar, const double *dphi_bar, double *eta_bar, double *phis_bar,
                         double *w_bar, void *stream);

/* VJP of fnpf_w_surface for the geometry of the last fnpf_geom: from w_s and
 * w_bar [n_s], adds to phi_bar (+=) [n_v] (top element layer only) and to
 * eta_bar (+=), h_bar (+=) [n_s] (the recovery divides by eta + h). */
fnpf_status fnpf_w_surface_vjp(fnpf_ctx ctx, const double *w_s, const double *w_bar, double *phi_bar,
                               double *eta_bar, double *h_bar, void *stream);

/* Adjoint Laplace solve (the operator is symmetric): A_II lambda_I = phi_bar_I,
 * lambda_S = 0, same options and stopping rule as fnpf_solve; lambda [n_v]
 * holds the initial guess on entry.  Synchronises the stream. */
fnpf_status fnpf_solve_adjoint(fnpf_ctx ctx, const double *phi_bar, double *lambda, const fnpf_solve_opts *opts,
                               fnpf_solve_info *info, void *stream);

/* VJP of the geometry dependence of the solve: adds d(-lambda^T A(eta, h) phi)
 * to eta_bar (+=) and h_bar (+=) [n_s], for the geometry of the last
 * fnpf_geom (lambda, phi [n_v]). */
fnpf_status fnpf_geom_vjp(fnpf_ctx ctx, const double *lambda, const double *phi, double *eta_bar, double *h_bar,
                          void *stream);

/* VJP of one fnpf_rk4_step taken from its tape: on entry eta_bar, phis_bar
 * [n_s] hold the adjoint of the step's output state; on exit, of its input
 * state; h_bar (+=) accumulates the adjoint of the depth.  Runs 4 adjoint
 * solves (opts) and recomputes the stage geometry; info (host, may be NULL)
 * gets one record per stage (index = stage).  t is the time at the start of
 * the step: calls for t, t - dt, t - 2 dt, ... form a sequence whose adjoint
 * solutions extrapolate the next call's initial guesses like
 * opts.extrapolate does for fnpf_rk4_step (a history of its own). */
fnpf_status fnpf_rk4_step_vjp(fnpf_ctx ctx, const double *h, double t, double dt, const double *tape,
                              double *eta_bar, double *phis_bar, double *h_bar, const fnpf_solve_opts *opts,
                              fnpf_solve_info *info, void *stream);

/* Copy the context's warm-start potential to/from phi[n_v] (device FP64);
 * phi == NULL in set_ resets it to zero.  Both also clear the step history
 * used by opts.extrapolate. */
fnpf_status fnpf_get_warm_start(fnpf_ctx ctx, double *phi, void *stream);
fnpf_status fnpf_set_warm_start(fnpf_ctx ctx, const double *phi, void *stream);

/* Synchronise `stream` and report a pending device-side error (FNPF_ERR_GEOM). */
fnpf_status fnpf_sync(fnpf_ctx ctx, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* FNPF_H */
