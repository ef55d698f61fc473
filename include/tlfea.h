/*
 * tlfea.h -- C ABI of the MI355X (gfx950) internal-force / tangent-stiffness
 * library for total-Lagrangian finite elements (arXiv 2604.10357, Part II).
 *
 * The library evaluates, for T10 tetrahedra and ANCF3443 shells with
 * Saint Venant-Kirchhoff or compressible Mooney-Rivlin stress plus optional
 * Kelvin-Voigt damping:
 *   - the internal force f_int(q, qdot)  (Sec. 4.3, Eqs. F_assembly,
 *     fint_local, fint_global, atomic_scatter);
 *   - the tangent  alpha * df/dq + beta * df/dqdot  scattered into a CSR
 *     matrix whose pattern is built once (Sec. 4.2; Sec. 4.4.2,
 *     Eq. tangent_block).  With (alpha, beta) = (h, 1) this is the Jacobian of
 *     f_int(q_n + h v, v) with respect to v, the tangent term of the Newton
 *     matrix H = M/h + h K_t + ... (Sec. 2, Eq. residual; Sec. 4.4.2,
 *     Eq. hessian);
 *   - vector-Jacobian products of f_int for reverse-mode differentiation.
 *
 * Conventions
 *   - Every call returns a status: TLFEA_OK (0) or a negative error code;
 *     tlfea_status_string() names it.  On error no output is written unless
 *     the description says otherwise.
 *   - Generalised coordinates are flat float64 arrays, DOF index
 *     3 * coef + d.  T10: coef = node.  ANCF3443: coef = 4 * node + k with
 *     k = 0..3 for (r, r_x, r_y, r_z).
 *   - Arrays named d_* are DEVICE pointers owned by the caller (e.g. the
 *     data_ptr of a torch tensor on the same GPU).  Arrays named h_* are host
 *     pointers.  The library copies what it keeps; the caller may free its
 *     arrays after a call returns.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Compute
 *     calls only enqueue work on it and return without synchronising; their
 *     outputs are valid once the stream reaches that point.  A mesh handle
 *     must not be used by two streams at the same time.
 *   - Outputs are overwritten (the library clears them on the stream); only
 *     tlfea_assemble_accumulate adds into what the caller passes.
 *   - The mesh handle owns device copies of connectivity, reference geometry,
 *     the CSR pattern and the slot map; tlfea_mesh_destroy frees them.
 */
#ifndef TLFEA_H
#define TLFEA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define TLFEA_OK 0
#define TLFEA_ERR_INVALID -1         /* bad argument: null pointer, size, index out of range */
#define TLFEA_ERR_UNSUPPORTED -2     /* element / material / rule / mesh feature not supported */
#define TLFEA_ERR_DEGENERATE -3      /* a reference element has det J0 <= 0 */
#define TLFEA_ERR_HIP -4             /* a HIP runtime call failed */
#define TLFEA_ERR_NOMEM -5           /* device allocation failed */
#define TLFEA_ERR_NO_PATTERN -6      /* call needs tlfea_build_csr_pattern first */
#define TLFEA_ERR_TOO_LARGE -7       /* nnz or an index does not fit int32 */

/* element types */
#define TLFEA_T10 1        /* 10-node quadratic tetrahedron, 5-point Keast rule (Sec. 4.3) */
#define TLFEA_ANCF3443 2   /* 4-node ANCF shell, nodes carry r, r_x, r_y, r_z (Sec. 4.3) */
#define TLFEA_ANCF3243 3   /* 2-node ANCF beam, nodes carry r, r_x, r_y, r_z; Gauss-Legendre 3x2x2 (Sec. 4.3) */

/* materials (Sec. 4.3, Stage 1) */
#define TLFEA_SVK 1           /* params = {E, nu, unused} */
#define TLFEA_MOONEY_RIVLIN 2 /* params = {mu10, mu01, kappa} */

/* arithmetic of the element kernels */
#define TLFEA_FP64 0   /* everything in float64 */
#define TLFEA_MIXED 1  /* stress, material tangent and K_e in float32; displacement gradient,
                          J - 1, J^(-2/3), J^(-4/3) and the volumetric coefficients in float64;
                          global f and CSR accumulation in float64 */

/* runtime flag bits (tlfea_get_runtime_flags) */
#define TLFEA_FLAG_INVERTED 1u    /* some quadrature point had det F <= 0 */
#define TLFEA_FLAG_NONFINITE 2u   /* some stress value was NaN or infinite */

typedef struct tlfea_mesh_s* tlfea_mesh_t;
typedef struct tlfea_batch_s* tlfea_batch_t;

typedef struct {
  int32_t elem_type;      /* TLFEA_T10 | TLFEA_ANCF3443 | TLFEA_ANCF3243 */
  int64_t n_coef;         /* number of coefficient vectors (T10: nodes; ANCF: 4 * nodes) */
  int64_t n_elem;
  const int32_t* h_conn;  /* T10: n_elem x 10 node ids, corners then edges (0,1),(1,2),(0,2),
                             (0,3),(1,3),(2,3); ANCF3443: n_elem x 4 node ids counter-clockwise
                             from parent corner (-1,-1); ANCF3243: n_elem x 2 node ids, the
                             element's parent axis running from the first to the second.
                             0-based. */
  const double* h_X;      /* n_coef x 3 reference coefficients */
  int32_t gl[3];          /* ANCF3443 Gauss-Legendre points per parent direction: {3,3,2} or
                             {4,4,3}; ANCF3243: {3,2,2}; ignored for T10 */
  double thickness;       /* ANCF3443 shell thickness H; ANCF3243 cross-section height H (along
                             r_z); ignored for T10 */
  int32_t material;       /* TLFEA_SVK | TLFEA_MOONEY_RIVLIN */
  double params[3];       /* see the material constants above */
  double kv_eta;          /* Kelvin-Voigt: S_v = 2 eta Edot + kv_lambda tr(Edot) I, P_v = F S_v */
  double kv_lambda;       /* both 0 disables damping */
  int32_t precision;      /* TLFEA_FP64 | TLFEA_MIXED */
  double width;           /* ANCF3243 cross-section width W (along r_y); ignored otherwise.  The
                             beam's length L is the reference distance of its two nodes and its
                             cross-section the rectangle W x H centred on the axis. */
} tlfea_mesh_desc;

/* Name of a status code (static string). */
const char* tlfea_status_string(int status);

/* Library version as major*10000 + minor*100 + patch. */
int tlfea_version(void);

/* Create a mesh on the current HIP device (Sec. 4.1: precompute once).
 * Copies conn and X to the device and computes the reference Jacobians J0,
 * det J0 and J0^-1 at every quadrature point (kept per element when an element
 * is affine).  Validates ids and element sizes; returns TLFEA_ERR_DEGENERATE
 * if any det J0 <= 0.  Synchronises the device.  *out is NULL on error. */
int tlfea_mesh_create(const tlfea_mesh_desc* desc, tlfea_mesh_t* out);

/* Free a mesh and everything it owns.  NULL is accepted. */
int tlfea_mesh_destroy(tlfea_mesh_t mesh);

/* Sizes: any pointer may be NULL.  nnz is -1 before the pattern is built. */
int tlfea_mesh_info(tlfea_mesh_t mesh, int64_t* n_dof, int64_t* n_elem, int64_t* nnz,
                    int32_t* n_en, int32_t* n_qp);

/* Replace the material (same meaning as the descriptor fields). */
int tlfea_mesh_set_material(tlfea_mesh_t mesh, int32_t material, const double params[3],
                            double kv_eta, double kv_lambda);

/* Switch between TLFEA_FP64 and TLFEA_MIXED element arithmetic. */
int tlfea_mesh_set_precision(tlfea_mesh_t mesh, int32_t precision);

/* Build the fixed CSR pattern of the DOF-level tangent and the slot map, once
 * (Sec. 4.2; Sec. 4.4.2).  Two coefficients are adjacent iff their nodes share
 * an element; every adjacent pair gives a full 3x3 block; rows are sorted.
 * Runs on the device (incidence lists, per-node sort-unique, prefix sums) and
 * synchronises.  Writes nnz (both triangles, structural zeros included).
 * Returns TLFEA_ERR_TOO_LARGE if nnz exceeds INT32_MAX and
 * TLFEA_ERR_UNSUPPORTED if a node is adjacent to more than 256 nodes (itself
 * included) or gathers more than 4096 candidate neighbours. */
int tlfea_build_csr_pattern(tlfea_mesh_t mesh, int64_t* nnz_out);

/* Copy the CSR pattern out: row_offsets[n_dof + 1], col_indices[nnz] (int32).
 * on_device != 0: destination pointers are device pointers (copy on `stream`
 * without synchronising); 0: host pointers (synchronous). */
int tlfea_get_csr_pattern(tlfea_mesh_t mesh, int32_t* row_offsets, int32_t* col_indices,
                          int32_t on_device, void* stream);

/* Upper triangle of the pattern (columns >= row: each row's suffix from its
 * diagonal on), the storage of a symmetric matrix given to a Cholesky solver
 * (the paper keeps the symmetric positive definite system in this form for its
 * factorization, Sec. 4.6).  Built on the device once (synchronises); nnz_upper
 * (may be NULL) receives its length.  A new full pattern drops it. */
int tlfea_build_upper_pattern(tlfea_mesh_t mesh, int64_t* nnz_upper);
/* Copy it out: row_offsets[n_dof + 1], col_indices[nnz_upper]; destination
 * semantics as in tlfea_get_csr_pattern.  TLFEA_ERR_INVALID before
 * tlfea_build_upper_pattern. */
int tlfea_get_csr_pattern_upper(tlfea_mesh_t mesh, int32_t* row_offsets, int32_t* col_indices,
                                int32_t on_device, void* stream);

/* Export the canonical DOF-level slot map for elements [elem_begin,
 * elem_begin + elem_count): slots[e][3a+i][3b+k] is the CSR position that
 * receives entry (i, k) of block (a, b) of element e, (3 n_en)^2 int32 per
 * element.  Destination semantics as in tlfea_get_csr_pattern. */
int tlfea_get_slot_map(tlfea_mesh_t mesh, int64_t elem_begin, int64_t elem_count, int32_t* slots,
                       int32_t on_device, void* stream);

/* f_int(q, qdot) -> d_f (n_dof float64).  d_qdot may be NULL (zero velocity).
 * Needs the pattern (tlfea_build_csr_pattern): the per-node reduction uses
 * its node-to-element incidence.  Each element's force is summed over its
 * points in one workgroup and left as one block of 3 mc values per (element,
 * node) incidence (float32 in mixed precision) in the mesh's work buffer; the
 * per-node sums then run in a fixed order, so repeated calls give the same
 * bits.  The first call that needs a larger work buffer allocates it and
 * synchronises; later calls do not allocate.
 * For the CSR-valued calls below, d_vals may be NULL exactly when the pattern
 * has no entries (a mesh without elements). */
int tlfea_internal_force(tlfea_mesh_t mesh, const double* d_q, const double* d_qdot, double* d_f,
                         void* stream);

/* Allocation-free form of tlfea_internal_force, for callers that cannot
 * allocate or free device memory during a call: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Same kernels, same
 * fixed summation order and therefore the same bits as tlfea_internal_force
 * on the same mesh and inputs; needs the pattern (TLFEA_ERR_NO_PATTERN
 * before).  Instead of the mesh's work buffer, the per-incidence force blocks
 * (n_elem * nodes per element * 3 * mc values: 4 bytes each in mixed
 * precision, 8 in float64) go to a work area compiled into the library,
 * TLFEA_NOALLOC_SCRATCH_BYTES per GPU, which each GPU the library runs on
 * holds until the process ends.  A mesh whose blocks exceed it is rejected
 * with TLFEA_ERR_TOO_LARGE before any work is enqueued (T10: up to 559,240
 * elements in mixed precision, 279,620 in float64).  Every block is written
 * before it is read, so the area needs no clearing between calls.  All calls
 * on one GPU share that GPU's area: calls that overlap in time on one GPU
 * (two streams, two host threads, two meshes) race and must be serialised by
 * the caller.  The call allocates nothing and frees nothing. */
#define TLFEA_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
int tlfea_internal_force_noalloc(tlfea_mesh_t mesh, const double* d_q, const double* d_qdot, double* d_f,
                                 void* stream);

/* Kernel forms of the tangent calls below (results equal up to rounding
 * order; Sec. 4.4.2, Eq. tangent_block): in mixed precision, a material
 * without Kelvin-Voigt damping has a symmetric tangent, and the element pass
 * then contracts only the slots i <= k of every point's tangent and stores the
 * others by transposition; the shell's contraction runs on the matrix cores.
 * Environment TLFEA_SYM_RECORDS=0 and TLFEA_MC_MFMA=0 (read once per process)
 * keep the full contraction and the vector form, for comparisons. */

/* CSR values of h * df/dq + df/dqdot = d f_int(q_n + h v, v) / dv -> d_vals (nnz). */
int tlfea_tangent(tlfea_mesh_t mesh, const double* d_q, const double* d_qdot, double h,
                  double* d_vals, void* stream);

/* CSR values of alpha * df/dq + beta * df/dqdot -> d_vals (nnz). */
int tlfea_tangent_ex(tlfea_mesh_t mesh, const double* d_q, const double* d_qdot, double alpha,
                     double beta, double* d_vals, void* stream);

/* Fused f_int and tangent (alpha, beta) = (h, 1) in one pass over the elements. */
int tlfea_assemble(tlfea_mesh_t mesh, const double* d_q, const double* d_qdot, double h,
                   double* d_f, double* d_vals, void* stream);

/* Fused f_int and tangent with explicit (alpha, beta). */
int tlfea_assemble_ex(tlfea_mesh_t mesh, const double* d_q, const double* d_qdot, double alpha,
                      double beta, double* d_f, double* d_vals, void* stream);

/* Same as tlfea_assemble_ex but ADDS into d_f and d_vals instead of
 * overwriting them (either may be NULL to skip it).  Lets a caller add
 * alpha * df/dq + beta * df/dqdot onto a matrix that already holds other terms
 * of the Newton matrix, e.g. M/h in H = M/h + h K_t + ... (Sec. 4.4.2,
 * Eq. hessian), without a separate clearing pass. */
int tlfea_assemble_accumulate(tlfea_mesh_t mesh, const double* d_q, const double* d_qdot, double alpha,
                              double beta, double* d_f, double* d_vals, void* stream);

/* Same as tlfea_assemble_ex, with the tangent written to the upper triangle
 * only (d_vals_upper: nnz_upper values on the pattern of
 * tlfea_build_upper_pattern).  Only for materials without Kelvin-Voigt
 * damping, whose tangent is symmetric (the hyperelastic dP/dF has major
 * symmetry); TLFEA_ERR_UNSUPPORTED otherwise, TLFEA_ERR_INVALID before
 * tlfea_build_upper_pattern.  Writes half the matrix values of the full call;
 * the computation is the full one. */
int tlfea_assemble_upper(tlfea_mesh_t mesh, const double* d_q, const double* d_qdot, double alpha,
                         double beta, double* d_f, double* d_vals_upper, void* stream);

/* The two passes of every assembly call, exposed so that a caller can put
 * other work between them (e.g. pass 1 of the next mesh) or time them:
 *   tlfea_assemble_points: per element and quadrature point, the constitutive
 *     update (Sec. 4.3, Stage 1), then, into the mesh's work buffer, one of:
 *     with the tangent in mixed precision, each element's rows of K_e
 *     (alpha dP/dF + beta dP/dFdot contracted over its points, Eq.
 *     tangent_block) and its force, one block per (element, node) incidence;
 *     with the tangent in float64, per point the stress and the tangent in
 *     parent coordinates with the quadrature volume folded in; without the
 *     tangent (want_tangent = 0), each element's force, one block per
 *     incidence.  Allocates the buffer when it is too small (synchronising).
 *   tlfea_assemble_nodes: per node, the sums of Eqs. fint_local / fint_global
 *     and Eq. tangent_block over the incident elements, written to d_f and / or
 *     d_vals (either may be NULL; d_vals needs want_tangent = 1); accumulate
 *     != 0 adds instead of overwriting.  Reads what the last
 *     tlfea_assemble_points of the same mesh left, any number of times;
 *     returns TLFEA_ERR_INVALID if that does not exist, lacks the tangent or
 *     used another precision.
 * tlfea_assemble_ex(...) is exactly tlfea_assemble_points(..., 1, s) followed
 * by tlfea_assemble_nodes(..., 0, s).
 * Reproducibility: calls with the tangent agree to rounding on repetition (a
 * few units in the last place of the largest value), not bit for bit, because
 * each node range adds its contributions in the order its waves deliver them;
 * an atomic scatter per entry (Sec. 4.3, Eq. atomic_scatter; Sec. 4.4.2)
 * behaves the same way.  The force alone (want_tangent = 0, and
 * tlfea_internal_force) is summed in a fixed order and repeats bit for bit. */
int tlfea_assemble_points(tlfea_mesh_t mesh, const double* d_q, const double* d_qdot, double alpha,
                          double beta, int32_t want_tangent, void* stream);
int tlfea_assemble_nodes(tlfea_mesh_t mesh, double* d_f, double* d_vals, int32_t accumulate,
                         void* stream);

/* Vector-Jacobian products of f_int for a cotangent w (n_dof):
 *   d_gq     = (df/dq)^T w        (n_dof; may be NULL)
 *   d_gqdot  = (df/dqdot)^T w     (n_dof; may be NULL)
 *   d_gparam = d(w . f)/d(p0, p1, p2, kv_eta, kv_lambda)  (5 float64; may be NULL);
 *              p = (E, nu, -) for SVK, (mu10, mu01, kappa) for Mooney-Rivlin.
 * The transpose of Eq. tangent_block (Sec. 4.4.2) applied to w, in float64
 * whatever the mesh precision.  Outputs are overwritten; only the products
 * asked for are formed (d_gqdot == NULL leaves out the velocity adjoint and its
 * work), and repeated calls give the same bits.  Needs the CSR
 * pattern (TLFEA_ERR_NO_PATTERN otherwise: its node ranges drive the per-node
 * sums); uses the mesh's work buffer, so a following tlfea_assemble_nodes
 * without a new tlfea_assemble_points returns TLFEA_ERR_INVALID. */
int tlfea_internal_force_vjp(tlfea_mesh_t mesh, const double* d_q, const double* d_qdot,
                             const double* d_w, double* d_gq, double* d_gqdot, double* d_gparam,
                             void* stream);

/* ---------------------------------------------------------------------------
 * Newton step pieces (meshes of affine elements: straight-sided T10, flat
 * rectangular ANCF3443 shells, straight prismatic ANCF3243 beams).
 * ------------------------------------------------------------------------- */
/* Build the consistent mass matrix once (Sec. 4.1: m_ij = int rho s_i s_j dV
 * over each element, M_e = [m_ij I_3], assembled over the elements): exact
 * integrals of the shape-function products (T10: quadratic x quadratic; ANCF:
 * Gauss-Legendre 4 points along the cubic directions, 2 across), float64, kept
 * on the device per pair of adjacent pattern nodes (ANCF: the 4 x 4 block of
 * their coefficient pairs).  density > 0.  Needs the CSR pattern
 * (TLFEA_ERR_NO_PATTERN); TLFEA_ERR_UNSUPPORTED for meshes with a non-affine
 * element (curved T10, warped shell, curved beam).  Synchronises; a new
 * pattern drops the mass. */
int tlfea_build_mass(tlfea_mesh_t mesh, double density);
/* M as DOF-level CSR values on the mesh pattern (nnz float64, device): the
 * row of coefficient a, component d holds m_ab at column (b, d) and 0 at the
 * other columns of each 3 x 3 block.
 * TLFEA_ERR_INVALID before tlfea_build_mass. */
int tlfea_get_mass(tlfea_mesh_t mesh, double* d_vals, void* stream);
/* f_int and the Newton matrix H = M/h + h K_t (Sec. 4.4.2, Eq. hessian,
 * without constraint terms), K_t being the tangent with (alpha, beta) =
 * (h, 1): H = M/h + h df/dq + df/dqdot, the Jacobian in v of Eq. grad_L at
 * q = q_n + h v, qdot = v.  Overwrites d_f (may be NULL) and d_vals (nnz).
 * The mass term enters the per-range sums of the second pass, so H costs one
 * write like K.  h > 0.  TLFEA_ERR_INVALID before tlfea_build_mass. */
int tlfea_assemble_newton(tlfea_mesh_t mesh, const double* d_q, const double* d_qdot, double h,
                          double* d_f, double* d_vals, void* stream);
/* The same Newton matrix in the upper-triangle storage a Cholesky solver takes
 * (Sec. 4.6): row r of d_vals_upper (nnz_upper float64) holds the entries of
 * H's row r from its diagonal on, on the pattern of tlfea_build_upper_pattern.
 * Only for materials without Kelvin-Voigt damping (H = M/h + h df/dq is then
 * symmetric); TLFEA_ERR_UNSUPPORTED otherwise, TLFEA_ERR_INVALID before
 * tlfea_build_mass or tlfea_build_upper_pattern.  d_f may be NULL. */
int tlfea_assemble_newton_upper(tlfea_mesh_t mesh, const double* d_q, const double* d_qdot, double h,
                                double* d_f, double* d_vals_upper, void* stream);
/* g = M (v - v_prev)/h + f_int - f_ext (Sec. 4.4.1, Eq. grad_L, without
 * constraint terms), n_dof float64 each, device; d_f_ext may be NULL (0).
 * A group of lanes per node over its mass row; overwrites d_g.  h > 0.  On a
 * T10 mesh the first call allocates a per-mesh buffer of n_dof doubles for
 * v - v_prev (later calls do not allocate; calls on one mesh must not overlap).
 * TLFEA_ERR_INVALID before tlfea_build_mass. */
int tlfea_newton_gradient(tlfea_mesh_t mesh, const double* d_v, const double* d_v_prev,
                          const double* d_f_int, const double* d_f_ext, double h, double* d_g,
                          void* stream);

/* First-order inner solver of one time step (Sec. 4.5, Alg. 2, without the
 * constraint and multiplier terms): AdamW with decoupled weight decay on
 * g(v) = M (v - v_n)/h + f_int(q_n + h v, v) - f_ext.  Per inner iteration
 * l = 1, 2, ...:  m = b1 m + (1 - b1) g;  s = b2 s + (1 - b2) g.g;
 * v = (1 - lr wd) v - lr (m / (1 - b1^l)) / (sqrt(s / (1 - b2^l)) + eps);
 * q = q_n + h v;  f_int(q, v);  g as above, starting from g = m = s = 0.
 * The loop stops after max_iters iterations or when, at a check (after the
 * first iteration and then every check_every iterations), ||g|| <= eps_in
 * (1 + ||v||) or ||g|| <= eps_rel ||g_0|| (g_0: the first gradient).
 * d_v holds the initial velocity on entry and the result on return; d_q
 * receives q_n + h v; d_f_ext may be NULL.  d_work: 4 n_dof float64 of
 * caller memory (moments, gradient, internal force; the gradient is left at
 * d_work + 2 n_dof).  iters_out / gnorm_out (host, may be NULL): iterations
 * run and the last ||g||.  Needs tlfea_build_mass; `stream` must not be the
 * legacy default stream (the iterations between checks are captured into a
 * HIP graph).  Synchronises at every check. */
typedef struct {
  double lr;           /* step size alpha */
  double beta1, beta2; /* moment decay rates, in [0, 1) */
  double eps;          /* > 0 */
  double weight_decay; /* lambda_wd >= 0 */
} tlfea_adamw_params;
int tlfea_adamw_solve(tlfea_mesh_t mesh, const tlfea_adamw_params* params, double h, const double* d_q_n,
                      const double* d_v_n, const double* d_f_ext, double* d_v, double* d_q, double* d_work,
                      int32_t max_iters, int32_t check_every, double eps_in, double eps_rel,
                      int32_t* iters_out, double* gnorm_out, void* stream);

/* The internal force and its VJP with the material constants read from device
 * memory instead of the mesh (Sec. 4.3, Stage 1; the VJP as for
 * tlfea_internal_force_vjp): d_params = (p0, p1, p2, kv_eta, kv_lambda), 5
 * float64 on the device, with p as in tlfea_mesh_desc for the mesh's material
 * kind (SVK: E, nu, unused; Mooney-Rivlin: mu10, mu01, kappa).  The mesh's own
 * constants are neither used nor changed, and no call synchronises with the
 * host: for differentiable callers whose constants live on the GPU (the torch
 * autograd wrapper).  Needs the pattern.  tlfea_internal_force_p takes the
 * force path of tlfea_internal_force (the same kernels and summation order);
 * d_gparam of the VJP holds d(w . f)/d(p0, p1, p2, kv_eta, kv_lambda) at
 * d_params. */
int tlfea_internal_force_p(tlfea_mesh_t mesh, const double* d_q, const double* d_qdot, const double* d_params,
                           double* d_f, void* stream);
int tlfea_internal_force_vjp_p(tlfea_mesh_t mesh, const double* d_q, const double* d_qdot, const double* d_params,
                               const double* d_w, double* d_gq, double* d_gqdot, double* d_gparam, void* stream);

/* Read (and synchronise on the mesh's last stream) the runtime flag bits,
 * then clear them. */
int tlfea_get_runtime_flags(tlfea_mesh_t mesh, uint32_t* flags);

/* ---------------------------------------------------------------------------
 * Launch shape of the per-node pass and its autotuning.
 * Not a step of the method: the shape decides how the nodes are cut into
 * ranges (each range is one workgroup whose CSR rows are one contiguous
 * segment held in LDS) and how many waves work on a range.  Every shape gives
 * the same result up to rounding order.  The default is {4, 768, 2048} for
 * T10 meshes created in mixed precision and {4, 768, 4096} otherwise
 * (environment TLFEA_GATHER_WAVES / TLFEA_RANGE_TASKS / TLFEA_RANGE_VALUES
 * override it when the pattern is built).
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t waves;        /* waves of 64 lanes per workgroup, 1 .. 8 */
  int32_t range_tasks;  /* cap on a range's tasks (9 per T10 incidence, 36 per ANCF) */
  int32_t range_values; /* cap on a range's CSR values + force rows, in float64 */
} tlfea_gather_shape;

/* Re-cut the mesh's node ranges for `shape` (a single node may exceed the
 * caps; a range never exceeds 64 nodes).  Needs the pattern
 * (TLFEA_ERR_NO_PATTERN); TLFEA_ERR_UNSUPPORTED, with the mesh unchanged, if a
 * range would need more than 96 KiB of LDS.  Synchronises the device. */
int tlfea_mesh_set_gather_shape(tlfea_mesh_t mesh, const tlfea_gather_shape* shape);
/* Current shape and number of ranges (either pointer may be NULL). */
int tlfea_mesh_get_gather_shape(tlfea_mesh_t mesh, tlfea_gather_shape* shape, int64_t* n_ranges);

/* Time tlfea_assemble(mesh, d_q, d_qdot, h, d_f, d_vals) for each shape of
 * the grid waves {2,4,8} x range_tasks {384,768,1536} x range_values
 * {2048,4096,8192} and for the shape in use (`reps` timed calls after one
 * warm-up, HIP events on `stream`), keep the fastest if it beats the shape in
 * use by at least 5 % (else keep that one), and leave the kept shape's result
 * in d_f / d_vals.  Shapes that do not fit are skipped.  chosen / ms_per_call (may be NULL) receive
 * the shape and its mean time per call.  reps in 1 .. 1000.  Synchronises;
 * meant to be called once, before a run of assemblies.  On an error the
 * previous shape is restored. */
int tlfea_mesh_autotune(tlfea_mesh_t mesh, const double* d_q, const double* d_qdot, double h,
                        double* d_f, double* d_vals, int32_t reps, void* stream,
                        tlfea_gather_shape* chosen, float* ms_per_call);

/* ---------------------------------------------------------------------------
 * Batched assembly of many independent bodies in one launch.
 * Each body keeps its own CSR (int32 within a body).  Body b owns
 * q/qdot/f[dof_off[b] .. dof_off[b+1]) and vals[nnz_off[b] .. nnz_off[b+1]).
 * All meshes must be of the same element type and have built patterns; they
 * must stay alive while the batch exists.  Materials and precision are read
 * from the meshes at tlfea_batch_create (mixed SVK / Mooney-Rivlin allowed),
 * together with the device arrays of their patterns: after
 * tlfea_build_csr_pattern, tlfea_mesh_set_material or tlfea_mesh_set_precision
 * (to another precision) on a member, every call on the batch (the graph and
 * loop forms alike) returns TLFEA_ERR_INVALID and writes nothing; create the
 * batch again.
 * ------------------------------------------------------------------------- */
int tlfea_batch_create(const tlfea_mesh_t* meshes, int32_t n_bodies, tlfea_batch_t* out);
int tlfea_batch_destroy(tlfea_batch_t batch);

/* Offsets (n_bodies + 1 each, host int64). */
int tlfea_batch_offsets(tlfea_batch_t batch, int64_t* dof_off, int64_t* nnz_off);

/* One launch over all bodies: f and tangent (h_b, 1) per body, h_b from the
 * device array d_h (n_bodies float64). */
int tlfea_batch_assemble(tlfea_batch_t batch, const double* d_q, const double* d_qdot,
                         const double* d_h, double* d_f, double* d_vals, void* stream);

/* Same as a loop of tlfea_assemble calls, one launch per body (reference path). */
int tlfea_batch_assemble_loop(tlfea_batch_t batch, const double* d_q, const double* d_qdot,
                              const double* d_h, double* d_f, double* d_vals, void* stream);

/* Schedule of the batched element-row launches (T10 bodies in mixed
 * precision; the persistent batched form).  persistent = 0: one
 * workgroup per element tile and per node range (the default).  persistent =
 * 1: grids of as many workgroups as the GPU holds at once, which take work
 * items from device counters: tiles of tile_elems (25 or 16) elements, full
 * tiles of the largest bodies first and partial tiles last, then node ranges
 * by decreasing work (longest-processing-time order).  Either schedule gives
 * the same results up to rounding order.  TLFEA_ERR_UNSUPPORTED for a batch
 * off the T10 element-row path (ANCF and float64 batches run per item).
 * get: grid_tiles / grid_ranges receive the workgroups launched per pass (any
 * pointer may be NULL). */
int tlfea_batch_set_schedule(tlfea_batch_t batch, int32_t persistent, int32_t tile_elems);
int tlfea_batch_get_schedule(tlfea_batch_t batch, int32_t* persistent, int32_t* tile_elems, int32_t* grid_tiles,
                             int32_t* grid_ranges);

/* The batch's own pass-2 launch shape (the bodies' shapes are not changed):
 * set, get and autotune as for a mesh, over the concatenated ranges of all
 * bodies.  The batch starts with the first body's shape.  A new shape drops
 * the captured graph of tlfea_batch_assemble (it is captured again at the
 * next call).  tlfea_batch_autotune times the uncaptured launch pair of
 * tlfea_batch_assemble on `stream` over every schedule (both forms above; on
 * the element-row path the persistent one with both tile sizes) and every
 * candidate shape, keeps the fastest (a change of schedule must gain at least
 * 5 %), and leaves its result in d_f / d_vals.  The choice is remembered for
 * the life of the process under the batch's signature (element type,
 * precision and every body's element and node counts): a batch created later
 * with the same signature starts with it. */
int tlfea_batch_set_gather_shape(tlfea_batch_t batch, const tlfea_gather_shape* shape);
int tlfea_batch_get_gather_shape(tlfea_batch_t batch, tlfea_gather_shape* shape, int64_t* n_ranges);
int tlfea_batch_autotune(tlfea_batch_t batch, const double* d_q, const double* d_qdot, const double* d_h,
                         double* d_f, double* d_vals, int32_t reps, void* stream, tlfea_gather_shape* chosen,
                         float* ms_per_call);

#ifdef __cplusplus
}
#endif
#endif /* TLFEA_H */
