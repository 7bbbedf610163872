/* ipibm.h -- C-ABI of the MI355X interaction-potential + immersed-boundary
 * Lagrangian step (Spandan et al., "A parallel interaction potential approach
 * coupled with the immersed boundary method for fully resolved simulations of
 * deformable interfaces and membranes").
 *
 * One call = one pass of a step of the method over a batch of triangulated
 * bodies: interaction-potential forces (Section 2.3), transfer between the
 * Lagrangian nodes and the staggered Eulerian grid (Section 2.2) and the
 * explicit node update (Section 2.3, Newton's second law per vertex).
 * Beside the step: the derivatives of its parts (forces JVP, interpolation
 * adjoint, reverse step, Taylor loss), the transfer at the triangle centroids
 * (MLS interpolation and spreading, direct forcing, external loads from
 * normal probes, centroid forces to the vertices; Section 2.2) and per-edge
 * weights on the spring and bending constants (Section 2.3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Positions X are double[N][3] (row-major, node-major), always FP64.
 * - "real" below is double for an IP_F64 plan and float for an IP_F32 plan.
 *   In IP_F32 plans edge vectors are formed from the FP64 positions before
 *   rounding, and the per-body volume, its reduction and the position update
 *   stay FP64.
 * - Node ids are int32 global indices into X.  Body b owns the nodes
 *   [node_off[b], node_off[b+1]), edges [edge_off[b], edge_off[b+1]) and faces
 *   [face_off[b], face_off[b+1]); every element of body b references only
 *   nodes of body b.
 * - Grid fields u (velocity) and f (force density) are real[3][nz][ny][nx],
 *   x fastest: component d lives on the MAC lattice d, u_x at
 *   (i, j+1/2, k+1/2) h, u_y at (i+1/2, j, k+1/2) h, u_z at (i+1/2, j+1/2, k) h
 *   (Section 2.1 staggered grid; offsets are our reading).  The box
 *   [0, nx h) x [0, ny h) x [0, nz h) is periodic in all directions.
 * - All pointers passed to compute entry points are DEVICE pointers unless
 *   marked "host".  The caller owns every array it passes; the plan owns only
 *   what it derives (connectivity copies, gather lists, workspace).
 * - Calls are asynchronous on `stream` (a hipStream_t, 0 = null stream).
 *   Argument errors return synchronously with IP_ERR_ARG and launch nothing.
 *   Device-detected conditions (degenerate element, non-finite value) set
 *   bits of the plan's status word, read by ip_plan_status().
 * - One plan may be used from one host thread at a time.  Calls on one plan
 *   that overlap in time (different streams) race on its workspace.
 */
#ifndef IPIBM_H
#define IPIBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ip_plan ip_plan;

typedef enum {
    IP_OK = 0,
    IP_ERR_ARG = -1,          /* invalid argument; nothing launched */
    IP_ERR_HIP = -2,          /* HIP runtime error (message in ip_last_error) */
    IP_ERR_DEGENERATE = -3,   /* returned by ip_plan_status only */
    IP_ERR_NONFINITE = -4,    /* returned by ip_plan_status only */
    IP_ERR_OOM = -5,          /* device allocation failed */
    IP_ERR_UNSUPPORTED = -6   /* valid request this build does not support */
} ip_status;

typedef enum { IP_F64 = 0, IP_F32 = 1 } ip_precision;

/* Status-word bits (ip_plan_status). */
#define IP_STATUS_DEGENERATE 0x1u  /* zero-length edge, zero-area face or hinge */
#define IP_STATUS_NONFINITE  0x2u  /* a non-finite force or velocity was produced */

/* Mesh of all bodies (Section 5 data structures: vertices of a face and the
 * four vertices of the two faces sharing an edge).  Everything is HOST memory,
 * read and copied during ip_plan_create only.
 *   faces[F][3]   triangle vertices, counter-clockwise seen from outside.
 *   edges4[E][4]  (v1, v2, v3, v4): (v1, v2) is the edge, v3 closes the face
 *                 (v1, v2, v3), v4 closes the face (v2, v1, v4); -1 marks a
 *                 missing face (open boundary: the edge keeps its spring but
 *                 has no bending hinge).
 *   closed[B]     1 = closed surface (volume potential applies), 0 = open.
 *   pinned[N]     1 = node never moves (may be NULL = none pinned).
 * Validation: offsets start at 0 and do not decrease; element nodes lie in
 * their body; v1 != v2; faces have three distinct nodes. */
typedef struct {
    int32_t n_bodies;
    const int64_t *node_off;
    const int64_t *edge_off;
    const int64_t *face_off;
    const int32_t *faces;
    const int32_t *edges4;
    const uint8_t *closed;
    const uint8_t *pinned;
} ip_mesh;

/* Periodic MAC grid: nx, ny, nz >= 3 cells of size h > 0. */
typedef struct {
    int32_t nx, ny, nz;
    double h;
} ip_grid;

/* Reference (stress-free) state, device arrays (Section 2.3: initial edge
 * lengths, angles between adjacent faces, triangle areas, body volumes).
 *   l0[E]      real   reference edge length
 *   cs0[E][2]  real   (cos theta0, sin theta0) of the signed reference
 *                     dihedral angle; (1, 0) on edges without a hinge
 *   A0[F]      real   reference triangle area
 *   V0[B]      double reference enclosed volume (closed bodies) */
typedef struct {
    const void *l0;
    const void *cs0;
    const void *A0;
    const double *V0;
} ip_reference;

/* Per-body constants, device double[B] each (Section 2.3: k_e, k_b, k_a, k_v
 * and the node mass m). */
typedef struct {
    const double *ks;
    const double *kb;
    const double *kA;
    const double *kV;
    const double *mass;
} ip_constants;

/* Launch-shape options of the fused step (0 in a field = the default):
 *   unit_nodes  bodies of at most this many nodes are one work unit (default
 *               and maximum: 4 x threads); larger bodies are split into
 *               patches;
 *   patch_owned owned nodes per patch (default 512, at least 16);
 *   tile_bytes  cap on the LDS tile region of a workgroup (default: all LDS
 *               left once the largest unit's arrays are placed; at least
 *               4096);
 *   threads     threads per workgroup of the fused kernel, with units of at
 *               most 4 x threads nodes: 768, 384, 256 or 128 for every unit; by
 *               default units above 1536 nodes run on 768 threads and the
 *               others on 384;
 *   wg_per_cu   workgroups per compute unit the tile of the smaller-unit
 *               launch (the only one when `threads` is set) is sized for:
 *               1 to 8 (default 2 for the 384-thread launch of the default
 *               split, else 1).  The LDS left per workgroup, once the
 *               largest unit's arrays are placed, is the tile; a unit whose
 *               cell box does not fit it spreads and interpolates directly
 *               against the grid.
 * The choice changes the speed, not the results beyond summation order. */
typedef struct {
    int32_t unit_nodes;
    int32_t patch_owned;
    int32_t tile_bytes;
    int32_t threads;
    int32_t wg_per_cu;
} ip_plan_options;

/* Build a plan: validates and copies the mesh, builds the node gather lists
 * and allocates workspace for N nodes.  `grid` may be NULL for plans that only
 * compute forces.  On success *plan is set; on failure it is left NULL. */
ip_status ip_plan_create(ip_plan **plan, const ip_mesh *mesh, const ip_grid *grid,
                         ip_precision precision);

/* ip_plan_create with launch-shape options (`options` may be NULL). */
ip_status ip_plan_create_ex(ip_plan **plan, const ip_mesh *mesh, const ip_grid *grid,
                            ip_precision precision, const ip_plan_options *options);

/* Release every resource of the plan (synchronizes the device). NULL is ok. */
ip_status ip_plan_destroy(ip_plan *plan);

/* Sizes: counts[0..3] = bodies, nodes, edges, faces. */
ip_status ip_plan_sizes(const ip_plan *plan, int64_t counts[4]);

/* Execution properties chosen at plan time:
 *   props[0] = 1 if ip_step runs the fused kernel (one workgroup per work
 *              unit), 0 if it runs the separate element, gather, transfer
 *              and update kernels;
 *   props[1] = nodes of the largest work unit;
 *   props[2] = LDS bytes of the per-unit grid tile;
 *   props[3] = threads per workgroup of the fused kernel;
 *   props[4] = number of work units: a body of at most props[3] x 4 nodes is
 *              one unit, a larger body is split into patches, each owning a
 *              compact set of its nodes and carrying every element that
 *              touches them (with the halo nodes those reach);
 *   props[5] = number of bodies split into patches. */
ip_status ip_plan_properties(const ip_plan *plan, int64_t props[6]);

/* Reference state from reference positions Xref[N][3] (Section 2.3 "initial
 * (reference) state").  Writes l0[E], cs0[E][2], A0[F] (real) and V0[B]
 * (double).  The signed angle follows the forces' convention: positive for a
 * convex fold, measured from the normal of face (v1, v2, v3) to that of
 * face (v2, v1, v4) about v2 - v1. */
ip_status ip_reference_from(ip_plan *plan, const double *Xref, void *l0, void *cs0,
                            void *A0, double *V0, void *stream);

/* Bind a reference to the plan: its arrays are copied (asynchronously on
 * `stream`; the caller may reuse them once the stream has passed this call)
 * into plan-owned storage.  Afterwards every entry point that takes an
 * ip_reference accepts NULL for "the bound reference".  For plans whose step
 * is fused (ip_plan_properties props[0] = 1) the bound copy is also packed
 * into per-element records, node ids local to the body with the element's
 * reference values (32 bytes per edge, 16 per face in FP64), ordered so that
 * every run of 64 elements touches distinct nodes where the mesh allows; the
 * fused step reads these records when given NULL, and the caller's arrays in
 * the caller's order otherwise (same results up to summation order).  Binding
 * again replaces the bound reference.  The first call allocates the storage
 * (IP_ERR_OOM on failure); later calls allocate nothing. */
ip_status ip_plan_bind_reference(ip_plan *plan, const ip_reference *ref, void *stream);

/* Bind per-edge weights on the spring and bending constants (Section 2.3:
 * on meshes of non-uniform triangles the edge stiffness varies edge by edge;
 * the paper points to an external model for it and does not print the rule,
 * so the weights come from the caller).  ew: device double[E][2], 16-byte
 * aligned, (w_s, w_b) for each edge in the mesh's edge order; edge e of body b then carries
 * ks[b] w_s[e] and kb[b] w_b[e] in every later call on the plan (forces,
 * energies, steps, their JVP and VJP; the constants' gradients are with
 * respect to the per-body ks, kb with the weights held fixed).  NULL unbinds
 * (every weight 1).  The weights are copied; the call synchronises `stream`
 * and returns IP_ERR_ARG, leaving the previous weights unbound, if any weight
 * is negative or not finite.  The first call allocates 16 bytes per edge and
 * per edge record (IP_ERR_OOM on failure); later calls allocate nothing. */
ip_status ip_plan_bind_edge_weights(ip_plan *plan, const double *ew, void *stream);

/* Interaction-potential forces at positions X (Section 2.3):
 *   W_e = 1/2 ks w_s (l - l0)^2           every edge
 *   W_b = kb w_b (1 - cos(theta - theta0)) every edge with two faces
 * (w_s, w_b: the bound per-edge weights, 1 when none are bound)
 *   W_a = 1/2 kA ((A - A0)/A0)^2 A0       every triangle
 *   W_v = 1/2 kV ((V - V0)/V0)^2 V0       every closed body
 * F = -grad(sum W) -> F[N][3] (real, overwritten).  V[B], A[B] (double,
 * may be NULL) receive each body's enclosed volume and area; W[B][4]
 * (double, may be NULL) the four energies (spring, bending, area, volume).
 * Element results are gathered into nodes through per-node lists; no
 * atomics, so F is bitwise reproducible. */
ip_status ip_forces(ip_plan *plan, const double *X, const ip_reference *ref,
                    const ip_constants *k, void *F, double *V, double *A, double *W,
                    void *stream);

/* ip_forces for callers that cannot allocate device memory during the call
 * or hold none of their own beside their inputs and outputs (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, kernels and results (bitwise) as ip_forces; the
 * element-slot workspace, and V and A when passed NULL, live in a static
 * device array of 64 MiB instead of the plan's buffers, so the call allocates
 * nothing and frees nothing.  The array holds 16 bytes per body (rounded up
 * to 256) plus 12 (FP64) or 6 (FP32) bytes per edge-slot/face-corner triple,
 * i.e. 3 (4E + 3F) reals: a plan needing more is refused with IP_ERR_ARG
 * before any launch (about 60 level-4 icosphere drops in FP64).  Each device
 * has one array, shared by every call on it and keeping the last call's
 * contents: calls that overlap on one device (several streams or host
 * threads) race and must be serialised by the caller. */
ip_status ip_forces_noalloc(ip_plan *plan, const double *X, const ip_reference *ref,
                            const ip_constants *k, void *F, double *V, double *A, double *W,
                            void *stream);

/* Interpolation of the staggered velocity to the nodes with the 3-point
 * regularised delta of Roma, Peskin & Berger (3x3x3 support, the support
 * domain of Section 2.2): U_d(X_l) = sum_k u_d[k] phi phi phi.
 * u: real[3][nz][ny][nx]; U: real[N][3] (overwritten).  Requires a grid. */
ip_status ibm_interp(ip_plan *plan, const double *X, const void *u, void *U, void *stream);

/* Spreading of nodal forces to the grid, the adjoint of ibm_interp up to h^3
 * (Section 2.2: total force conserved): f_d[k] += sum_l F_{l,d} phi phi phi / h^3.
 * F: real[N][3]; f: real[3][nz][ny][nx], ACCUMULATED (caller zeroes it).
 * Uses device atomics on f: the summation order is not fixed. */
ip_status ibm_spread(ip_plan *plan, const double *X, const void *F, void *f, void *stream);

/* Moving-least-squares transfer at the triangle centroids (Section 2.2: the
 * centroids are the Lagrangian markers; the MLS equations with the linear
 * basis [1, x, y, z]; the exponential weight on the 3x3x3 support of
 * threshold 1.5 h).  Marker l is the centroid of face l, for every face of
 * the plan's mesh.  Readings of the paper: the weight is a product over the
 * axes, W_k = prod_a w(|x_a - x^k_a| / (1.5 h)), w(r) = exp(-(r/alpha)^2)
 * for r <= 1 (the paper's r_i is the support size in direction i); the
 * moment matrix is A = sum_k W_k p(x^k) p(x^k)^T.  alpha > 0 is the shape
 * parameter, which the paper does not fix.
 * ibm_interp_mls: U[F][3] (real, overwritten), component d interpolated from
 * lattice d of u (real[3][nz][ny][nx]): U_{l,d} = sum_k phi_k u_d[k], with
 * phi^T = p(x)^T A^{-1} B.  Requires a grid; alpha must be positive and
 * finite.  A non-finite shape function sets IP_STATUS_NONFINITE. */
ip_status ibm_interp_mls(ip_plan *plan, const double *X, const void *u, double alpha, void *U,
                         void *stream);

/* Spreading of the marker force densities Fm[F][3] (real) with the same
 * shape functions and the force-conserving factor of Section 2.2:
 * f_d[k] += c_l phi_k Fm_{l,d}, c_l = dV_l / sum_k phi_k dV^k, dV_l = A_l h_l,
 * h_l = (1/3) sum_k phi_k (dx + dy + dz), dV^k = h^3, A_l the face area, so
 * that sum_k f_d[k] h^3 = sum_l dV_l Fm_{l,d}.  f: real[3][nz][ny][nx],
 * ACCUMULATED (caller zeroes it), device atomics (summation order not
 * fixed).  Requires a grid; alpha positive and finite. */
ip_status ibm_spread_mls(ip_plan *plan, const double *X, const void *Fm, double alpha, void *f,
                         void *stream);

/* Direct-forcing immersed-boundary force at the centroid markers (Section
 * 2.2): F_l = (Vb_l - U_l) / dt, with U_l the MLS interpolation of u at the
 * centroid of face l (as ibm_interp_mls) and Vb_l the desired velocity of the
 * marker; F is spread to f with the same shape functions and the factor c_l
 * (as ibm_spread_mls), in one pass that computes each marker's shape
 * functions once.  Vb: real[F][3]; u: real[3][nz][ny][nx]; Fm: real[F][3]
 * receives F (may be NULL); f: real[3][nz][ny][nx], ACCUMULATED (caller
 * zeroes it), device atomics.  alpha and dt positive and finite. */
ip_status ibm_direct_forcing_mls(ip_plan *plan, const double *X, const void *Vb, const void *u,
                                 double alpha, double dt, void *Fm, void *f, void *stream);

/* External (hydrodynamic) loads on the faces by normal probes (Section 2.2).
 * From each face centroid x_c a probe of length h runs along the unit normal
 * n (counter-clockwise corner order seen from outside): one outward probe on
 * closed bodies, one on each side of open ones.  At a probe end y = x_c + s h n
 * (s = +1 or -1): p = P(y) + s h acc.n with P the MLS value of the
 * cell-centred pressure (lattice points at cell centres), G_ij = du_i/dx_j
 * the gradient of the MLS linear fit of lattice i at y, tau = mu (G + G^T);
 * Fext = sum over the probes of s (-p n + tau n) A_f (for an open body, the
 * jump -(p+ - p-) n + (tau+ - tau-) n).  Readings of the paper: the probe
 * length is h (the mean local grid size of a uniform grid); the velocity
 * gradient is that of the local MLS linear fit; the acceleration correction
 * carries the probe's side s.  u: real[3][nz][ny][nx]; p: real[nz][ny][nx];
 * acc: real[F][3] marker acceleration Du/Dt (may be NULL: zero); Fext:
 * real[F][3] (overwritten).  alpha positive, mu >= 0, both finite.  A
 * zero-area face has no normal: its load is 0 and IP_STATUS_DEGENERATE is
 * set (IP_STATUS_NONFINITE for a non-finite normal). */
ip_status ibm_probe_loads(ip_plan *plan, const double *X, const void *u, const void *p,
                          const void *acc, double alpha, double mu, void *Fext, void *stream);

/* Centroid forces to the vertices (Section 2.3): Fn[n] = (1/3) sum of Fc[f]
 * over the faces f of vertex n.  Fc: real[F][3]; Fn: real[N][3]
 * (overwritten).  A gather over the plan's per-node lists: no atomics,
 * bitwise reproducible. */
ip_status ip_centroid_to_nodes(ip_plan *plan, const void *Fc, void *Fn, void *stream);

/* One explicit step (Section 2.3 Newton update, loosely coupled; the external
 * load is the immersed-boundary reaction m (U - Xdot)/dt of Section 2.2's
 * direct forcing, so that Xdot = U + (dt/m) F):
 *   F = forces(X), U = interp(u, X), f += spread(F, X),
 *   X <- X + dt U + (dt^2/m_b) F       for nodes that are not pinned.
 * X is updated in place.  V[B], A[B] (may be NULL) receive the volumes and
 * areas at the old positions.  f may be NULL (no spreading). */
ip_status ip_step(ip_plan *plan, double *X, const ip_reference *ref, const ip_constants *k,
                  const void *u, void *f, double dt, double *V, double *A, void *stream);

/* ---- derivatives (IP_F64 plans; IP_ERR_UNSUPPORTED otherwise) ---- */

/* Directional derivative of the forces: dF = (dF/dX) dX, where F is the force
 * of ip_forces.  F = -grad W, so dF/dX is the negated Hessian of the total
 * potential: symmetric, and this product is also the vector-Jacobian product.
 * Evaluated in forward mode (dual numbers) through the element code, with the
 * volume term's rank-one part from the tangent of each body's volume.
 * X, dX, dF: double[N][3] (dF overwritten).  Deterministic (gather lists). */
ip_status ip_forces_jvp(ip_plan *plan, const double *X, const double *dX,
                        const ip_reference *ref, const ip_constants *k, double *dF,
                        void *stream);

/* Reverse mode of one ip_step.  With the update X' = X + M (dt U(X) + dt^2/m
 * F(X; k)), M = not-pinned mask, and the adjoint lam_next = dL/dX', writes
 *   lam = lam_next + dt J_U(X)^T P + (dt^2/m) (dF/dX) P,   P = M lam_next,
 * and ACCUMULATES
 *   gk[s][b] += (dt^2/m_b) sum_{l in b} (F_s,l / k_s) . P_l   (s = spring,
 *               bending, area, volume; gk is double[4][B], may be NULL)
 *   gu       += dt h^3 spread(P)   (double[3][nz][ny][nx], may be NULL; the
 *               adjoint of interpolation is spreading).
 * X is the position at which the forward step was taken (a checkpoint).
 * lam may alias lam_next.  On plans with a fused step (ip_plan_properties
 * props[0] = 1) this runs as one fused kernel per work unit over the same
 * packed element records (accumulations in a run-dependent order) and
 * allocates nothing; otherwise the first call allocates a workspace of
 * 16 (E + F) bytes and the element kernels run separately. */
ip_status ip_step_vjp(ip_plan *plan, const double *X, const ip_reference *ref,
                      const ip_constants *k, const double *u, double dt, const double *lam_next,
                      double *lam, double *gk, double *gu, void *stream);

/* Adjoint of the interpolation ibm_interp (Section 2.2 transfer; the
 * backward pass of the calibration workload): for a cotangent dU[N][3] on the
 * interpolated velocities U = I(X) u,
 *   gX[l] = sum_d dU[l][d] dU_d/dX_l  (J_U^T dU: the 3-point delta and its
 *           derivative per axis; overwritten; may be NULL),
 *   gu_d[k] += sum_l dU[l][d] w_k(X_l)  (the transpose of interpolation,
 *           i.e. spreading without the 1/h^3; accumulated, the caller zeroes
 *           it; may be NULL).
 * X, dU, gX: double[N][3]; u, gu: double[3][nz][ny][nx].  IP_F64 plans only
 * (IP_ERR_UNSUPPORTED otherwise); gu is summed with device atomics, so it is
 * reproducible to rounding, not bitwise. */
ip_status ibm_interp_vjp(ip_plan *plan, const double *X, const double *u, const double *dU,
                         double *gX, double *gu, void *stream);

/* Taylor deformation of every body (Section 3.1 measure D = (L - B)/(L + B)):
 * L^2 and B^2 are the largest and smallest eigenvalues of the node covariance
 * C = (1/n) sum (x - c)(x - c)^T (our reading of the semi-axes).  D[B] may be
 * NULL.  With Dstar[B] given, also loss[b] = (D_b - Dstar_b)^2 and the
 * gradient gX[N][3] of sum_b loss[b] (overwritten).  All device double. */
ip_status ip_taylor(ip_plan *plan, const double *X, const double *Dstar, double *D,
                    double *loss, double *gX, void *stream);

/* Wait for the plan's work on `stream`, read and clear the status word.
 * Returns IP_OK, IP_ERR_DEGENERATE or IP_ERR_NONFINITE; *flags (may be NULL)
 * receives the raw bits. */
ip_status ip_plan_status(ip_plan *plan, void *stream, uint32_t *flags);

/* Message of the last error on the calling thread ("" if none). */
const char *ip_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* IPIBM_H */
