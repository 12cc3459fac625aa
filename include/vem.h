/*
 * vem.h - C ABI of the MI355X (gfx950) mixed virtual element solver.
 *
 * The library solves the saddle-point system that the mixed virtual element
 * method produces for the Darcy / mixed Poisson problem on a 3D polyhedral
 * mesh (Dassi & Scacchi, "Parallel solvers for virtual element
 * discretizations of elliptic equations in mixed form"):
 *
 *     nu u + grad p = 0,   div u = f   in Omega,   p = p_D on dOmega,
 *
 * or, with vem_set_boundary(h, VEM_BC_FLUX), u.n = u_N on dOmega and a pressure
 * of zero mean (the paper's model problem, Section 3),
 * discretised as in Sections 4.1-4.3 of the paper (face normal-flux moments,
 * L2 projector built through integration by parts, stabilised local forms)
 * and assembled in the symmetric form (Section 5, matrix with blocks A, B^T,
 * B, -C, here with C = 0 and A = M):
 *
 *     [ M  B^T ] [u]   [  g ]       B = -B_div,
 *     [ B   0  ] [p] = [ -F ],      g_i = -int_{dOmega} p_D phi_i . n.
 *
 * The system is solved by right-preconditioned restarted flexible GMRES with
 * one of the paper's two block-diagonal preconditioners (Section 5, eqs.
 * block_schur and block_diag):
 *   VEM_PREC_SCHUR: diag(M)^{-1} on the flux block, an inner Jacobi-CG solve
 *                   of S = B diag(M)^{-1} B^T on the pressure block;
 *   VEM_PREC_REG:   an inner Jacobi-CG solve of M + B^T B / gamma on the flux
 *                   block, gamma^{-1} I on the pressure block, gamma = h^2 with
 *                   h the mean cell diameter (eq. meshSize).
 *
 * Conventions for every entry point:
 *   - Every function returns a vem_status: 0 = success, > 0 = warning with
 *     valid outputs, < 0 = error with the outputs left untouched.  No C++
 *     exception crosses the ABI.  vem_last_error() gives the message of the
 *     last failure on a handle.
 *   - The caller owns every pointer it passes; the library owns only the
 *     device memory it allocates internally, released by vem_destroy().
 *   - "device" pointers are HIP device allocations on the handle's device;
 *     "host" pointers are ordinary host memory.  Device buffers must not be
 *     aliased unless stated.
 *   - All device work is enqueued on the stream given to vem_create();
 *     functions that return host-visible results synchronise that stream.
 *   - One handle must not be used by two host threads at once.
 *   - Index arrays are int32; sizes are limited to 2^31 - 1 entries.
 */
#ifndef VEM_H
#define VEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vem_ctx* vem_handle;
typedef int vem_status;

enum {
  VEM_OK = 0,
  VEM_NOT_CONVERGED = 1, /* tolerance not reached within maxit: best iterate written */
  VEM_EINVAL = -1,       /* invalid argument or call order */
  VEM_EBADMESH = -2,     /* inconsistent mesh (bad index, open cell, zero area/volume, ...) */
  VEM_ENOMEM = -3,       /* device allocation failed or size limit exceeded */
  VEM_EHIP = -4,         /* HIP runtime error */
  VEM_EBREAKDOWN = -5,   /* Krylov breakdown that could not be recovered */
  VEM_ENAN = -6          /* NaN or Inf met in the solve */
};

enum { VEM_MEM_HOST = 0, VEM_MEM_DEVICE = 1 };

/* Element families.  VEM_LO: the lowest-order member of the paper's face
 * space (Section 4.1) - one normal-flux moment per face, divergence and
 * pressure constant per cell.  VEM_PAPER: the paper's order-k element
 * (Sections 4.1-4.3: face space P_k with (k+1)(k+2)/2 moments per face,
 * gradient and cross interior moments, divergence and pressure P_{k-1}),
 * k = 1, 2, 3. */
enum { VEM_LO = 0, VEM_PAPER = 1 };

enum { VEM_PREC_SCHUR = 0, VEM_PREC_REG = 1, VEM_PREC_NONE = 2 };
/* Boundary data (vem_set_boundary).  VEM_BC_PRESSURE: the pressure p_D is given on the whole
 * boundary (natural in mixed form, the default).  VEM_BC_FLUX: the normal flux u.n = u_N is given on
 * the whole boundary and the pressure has zero mean, the paper's model problem (Section 3, eq.
 * mod_prob_eq; its DOF counts add one multiplier for the mean). */
enum { VEM_BC_PRESSURE = 0, VEM_BC_FLUX = 1 };

/* Arithmetic of the inner preconditioner solves.  VEM_FP64: everything in
 * FP64.  VEM_MIXED: the inner Jacobi-CG of either block preconditioner runs
 * with FP32 vectors and FP32 matrix values (dot products accumulated in
 * FP64): the one-kernel pipelined iteration when inner_maxit <= 64, the
 * classical two-kernel one otherwise.  The outer FGMRES, its residuals,
 * Gram-Schmidt and all assembly stay FP64, so the outer tolerance is met in
 * FP64 (flexible GMRES absorbs the FP32 preconditioner as it absorbs any
 * inexact inner solve). */
enum { VEM_FP64 = 0, VEM_MIXED = 1 };

/* Form of the inner Jacobi-preconditioned iteration.  VEM_INNER_PIPELINED (the default): CG, one
 * kernel per iteration (Ghysels-Vanroose recurrences).  VEM_INNER_CLASSICAL: CG with the textbook
 * recurrences in two kernels per iteration; slower, but its residual stays closer to the true one
 * on very ill-conditioned blocks (the paper's order-3 element, where the pipelined recurrences
 * stall the outer solve).  VEM_INNER_CHEBYSHEV: the Chebyshev iteration on D^{-1}A over the
 * interval [cheb_lo * hi, hi], hi the Gershgorin bound of D^{-1}A: a fixed polynomial of degree
 * inner_maxit, one kernel per degree and no reductions (inner_tol and use_graphs do not apply). */
enum { VEM_INNER_PIPELINED = 0, VEM_INNER_CLASSICAL = 1, VEM_INNER_CHEBYSHEV = 2 };

/* Preconditioner of Block-Reg's inner CG on A_gamma = M + B^T B / gamma (Section 5, eq.
 * block_diag, where the paper applies one algebraic multigrid cycle).  VEM_REG_JACOBI: diag(A_gamma)
 * (the inner_form and use_graphs options apply).  VEM_REG_SCHWARZ: additive Schwarz over the mesh
 * edges.  Each patch is the set of DOFs of the faces around one edge; these patches hold the local
 * divergence-free fluxes that dominate the small eigenvalues of A_gamma, which a diagonal
 * preconditioner never sees.  For the order-k element the interior DOFs of each cell are first
 * condensed exactly (static condensation), and the CG runs on the face DOFs; two kernels per
 * iteration; inner_form and use_graphs are ignored.  Limits: at most 80 DOFs per patch (faces around
 * one edge times face DOFs: 8 faces at k = 3, 13 at k = 2) and 160 faces sharing an edge with one
 * face; a mesh beyond them makes the Block-Reg solve fail with VEM_EINVAL (use VEM_REG_JACOBI). */
enum { VEM_REG_JACOBI = 0, VEM_REG_SCHWARZ = 1 };

/* matrices for vem_export_csr: the saddle matrix, S, A_gamma; the Block-Reg Schwarz preconditioner's
 * face system (A_gamma with the cell interiors condensed; A_gamma itself at the lowest order) and its
 * operator P = sum_e R_e^T F_e^{-1} R_e over the edge patches, both on the face DOFs. */
enum { VEM_MAT_K = 0, VEM_MAT_SCHUR = 1, VEM_MAT_REG = 2, VEM_MAT_REG_FACE = 3, VEM_MAT_REG_SCHWARZ = 4 };

typedef struct {
  int64_t n_vertices, n_faces, n_cells;
  int64_t n_u;       /* flux unknowns (face moments, then interior moments) */
  int64_t n_p;       /* pressure unknowns (moments, cell by cell) */
  int64_t n;         /* n_u + n_p */
  int64_t nnz_K;     /* saddle matrix [M B^T; B 0] */
  int64_t nnz_schur; /* S = B diag(M)^{-1} B^T */
  int64_t nnz_reg;   /* M + B^T B / gamma */
  int64_t n_qp_cell; /* volume quadrature points (load f) */
  int64_t n_qp_face; /* boundary-face quadrature points (p_D, or the flux field with VEM_BC_FLUX) */
  int32_t load_points; /* quadrature points per direction of the load rule */
  int32_t max_cell_faces;
  double h;          /* mean cell diameter (eq. meshSize) */
  double gamma;      /* default Block-Reg parameter h^2 */
  int64_t n_face_dofs; /* flux unknowns on faces (the first n_face_dofs of u) */
} vem_sizes;

typedef struct {
  int32_t precond;     /* VEM_PREC_* */
  int32_t restart;     /* FGMRES restart length m, 1..32 */
  int32_t maxit;       /* maximum outer iterations */
  int32_t use_x0;      /* nonzero: u, p hold the initial guess */
  double tol;          /* stop when ||b - K x||_2 <= tol ||b||_2 */
  double inner_tol;    /* relative tolerance of the inner Jacobi-CG (preconditioned residual) */
  int32_t inner_maxit; /* iteration cap of one inner solve.  A cap <= 64 enqueues all of them
                          without host polling (launches after the stop test return at once) */
  int32_t inner_check; /* inner iterations enqueued between convergence checks (cap > 64) */
  double gamma;        /* Block-Reg gamma; <= 0 selects h^2 */
  int32_t precision;   /* VEM_FP64 or VEM_MIXED */
  int32_t use_graphs;  /* nonzero: replay the inner-CG iterations as a captured HIP graph (same
                          kernels and arguments, identical results; a cap > 64 may be passed
                          by up to 7 iterations, as graphs run 8 at a time).  Default 0: on
                          gfx950 each replay boundary leaves the GPU idle for about 8 us,
                          more than the host's launch cost it saves */
  int32_t inner_form;  /* VEM_INNER_PIPELINED (default) or VEM_INNER_CLASSICAL */
  int32_t reg_inner;   /* Block-Reg inner preconditioner: VEM_REG_SCHWARZ (default) or VEM_REG_JACOBI */
  double cheb_lo;      /* VEM_INNER_CHEBYSHEV: lower end of the interval over the upper, in (0, 1);
                          <= 0 selects 1/200 */
} vem_solve_opts;

typedef struct {
  int32_t iterations;       /* outer FGMRES iterations */
  int32_t restarts;         /* completed restart cycles */
  int64_t inner_iterations; /* total inner CG iterations */
  double relres;            /* true ||b - K x|| / ||b|| of the returned iterate */
  double solve_ms;          /* wall time of vem_solve */
  int32_t status;
} vem_solve_info;

/* Fill opts with defaults: Block-Schur, m = 30, maxit = 5000, tol = 1e-8,
 * inner_tol = 1e-6, inner_maxit = 5000, inner_check = 32, gamma = h^2, FP64,
 * graphs off, pipelined inner CG. */
void vem_solve_opts_default(vem_solve_opts* opts);

/* Create a handle bound to the current HIP device and to `stream`
 * (a hipStream_t; NULL = the default stream).  The handle carries one instance of the paper's
 * discrete problem (Section 4.3, eq. mod_prob_eqDisc) and its solver state.  Errors: VEM_EINVAL
 * (h NULL), VEM_ENOMEM, VEM_EHIP. */
vem_status vem_create(vem_handle* h, void* stream);
vem_status vem_destroy(vem_handle h);

/* Set the polyhedral mesh Omega_h (Section 2: polyhedra P with planar polygonal faces; the
 * paper's Section 4.4 meshes are of this kind), copied in; the caller may free its arrays on
 * return.  xyz[nv*3]: vertex coordinates.  face_ptr[nf+1], face_vtx: the
 * vertex loop of each planar convex face, counter-clockwise about the face's
 * global normal n_f.  cell_ptr[nc+1], cell_face, cell_face_sign: the faces of
 * each cell and sigma = +1 if n_f points out of the cell, -1 otherwise.  Every
 * face must bound one cell (boundary) or two cells of opposite sign.  All
 * arrays are host or device memory according to mem_kind (device offsets are
 * checked on the device, never copied to the host).  Errors: VEM_EINVAL
 * (sizes), VEM_EBADMESH (offset arrays not starting at 0 or decreasing,
 * indices out of range, a face used twice with one sign, a face of no cell,
 * zero area, non-positive volume). */
vem_status vem_set_mesh(vem_handle h, int64_t nv, const double* xyz, int64_t nf, const int32_t* face_ptr,
                        const int32_t* face_vtx, int64_t nc, const int32_t* cell_ptr, const int32_t* cell_face,
                        const int8_t* cell_face_sign, int mem_kind);

/* Build geometry, local matrices (nu = 1) and the sparse patterns.
 * family: VEM_LO (k ignored) or VEM_PAPER (k = 1, 2, 3).  Flux unknowns are
 * ordered face by face (the face moments, w.r.t. the global normal and the
 * face frame: origin at the face centroid, e1 along the longest loop edge,
 * e2 = n_f x e1), then cell by cell (gradient moments, then cross moments:
 * x part, y part, z part; multi-indices graded, x power then y power
 * descending); pressure unknowns cell by cell.  load_points: points per direction of the
 * conical-product rule used for f and p_D (1..6; degree 2n-1).  The
 * coefficient is set to nu = 1 and the right-hand side to zero. */
vem_status vem_discretize(vem_handle h, int family, int k, int load_points);

/* Sizes of the discretisation (DOF counts of Section 4.1's spaces: per face dim P_k(f) moments,
 * per cell dim P_{k-1} - 1 + dim G_k^oplus interior moments and dim P_{k-1} pressure moments; the
 * lowest order 1, 0, 1), matrix sizes, quadrature point counts, h and gamma = h^2 (Section 5,
 * eq. meshSize).  out: host.  Errors: VEM_EINVAL before vem_discretize. */
vem_status vem_get_sizes(vem_handle h, vem_sizes* out);

/* Write the quadrature points at which the caller evaluates f and p_D (the loads of Section 4.3,
 * which the paper notes depend only on the quadrature formulas used; device buffers): qp_cell[3*n_qp_cell] and qp_face[3*n_qp_face] (either
 * may be NULL to skip), as structures of arrays: all x coordinates, then all
 * y, then all z.  Points are ordered cell by cell, then by the tetrahedra
 * (x_ref, v0, v_a, v_{a+1}) of each face, then by the reference points;
 * boundary-face points follow the boundary faces in face order. */
vem_status vem_get_quadrature(vem_handle h, double* qp_cell, double* qp_face);

/* nu = 1/K per cell (device or host, n_cells doubles, all > 0; copied in).
 * The flux block M (M_P is proportional to nu_P, Section 4.3) and the
 * preconditioner matrices are rebuilt from the stored coefficient-free local
 * matrices by the next call that uses them (vem_solve, vem_apply,
 * vem_export_csr, vem_time_kernel), each only when that call needs it (S for
 * Block-Schur, M + B^T B / gamma for Block-Reg); the local projectors are not
 * recomputed.  Errors: VEM_EINVAL if a value is not positive and finite
 * (checked on the device; the previous coefficient stays in place). */
vem_status vem_set_coefficient(vem_handle h, const double* nu);

/* Multi-field batch: nbatch coefficient fields nu[nbatch * n_cells] (field b at offset b * n_cells;
 * host or device; copied in, every value checked positive and finite on the device), for
 * vem_solve_batch.  The blueprint's nbatch of the coefficient (Section 4.3: M_P = nu_P M1_P, so a field
 * only rescales the stored coefficient-free local matrices).  Replaces any earlier batch; the handle's
 * own coefficient (vem_set_coefficient) is unchanged.  Errors: VEM_EINVAL (nothing stored). */
vem_status vem_set_coefficient_batch(vem_handle h, int64_t nbatch, const double* nu);

/* nbatch right-hand sides from point values, for vem_solve_batch: f_qp[nbatch * n_qp_cell] and
 * pD_qp[nbatch * n_qp_face] (NULL: p_D = 0), field b at offset b times the point count (device).
 * Each is loaded as vem_set_rhs loads one; the handle's own right-hand side is unchanged.  Pressure
 * boundary data only.  Errors: VEM_EINVAL. */
vem_status vem_set_rhs_batch(vem_handle h, int64_t nbatch, const double* f_qp, const double* pD_qp);

/* Solve nbatch systems of eq. mod_prob_eqDisc: system b takes coefficient field b of
 * vem_set_coefficient_batch (or the handle's coefficient if no batch of fields is set) and right-hand
 * side b of vem_set_rhs_batch (or its single right-hand side if one was set, or the handle's
 * [g; -F] if none).  u[nbatch * n_u], p[nbatch * n_p]: device, system b at offset b * n_u and b * n_p.
 * info[nbatch] (host, may be NULL).  The systems are solved one after another on the handle's stream
 * with the same options; each field rebuilds the coefficient-dependent values (K, and S or A_gamma with
 * its preconditioner) from the stored local matrices.  The handle's coefficient is restored on return.
 * Returns the first error, else the largest warning (VEM_NOT_CONVERGED if any system missed tol).
 * Errors: VEM_EINVAL when neither nbatch fields nor nbatch right-hand sides are set, or their counts
 * differ from nbatch. */
vem_status vem_solve_batch(vem_handle h, const vem_solve_opts* opts, int64_t nbatch, double* u, double* p,
                           vem_solve_info* info);

/* Right-hand side [g; -F] of eq. mod_prob_eqDisc from point values (device): F_P = int_P f psi
 * (Section 4.3) from f_qp[n_qp_cell] at the points of vem_get_quadrature, and the boundary term
 * g = -int_{dOmega} p_D phi.n from pD_qp[n_qp_face] (NULL means p_D = 0).  Errors: VEM_EINVAL
 * (before vem_discretize, or with flux boundary data); non-finite values are not checked here, a
 * later vem_solve reports them (VEM_ENAN). */
vem_status vem_set_rhs(vem_handle h, const double* f_qp, const double* pD_qp);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): vem_set_rhs with the same arguments, kernels and result,
 * that calls no hipMalloc, hipFree or allocating library routine.  Its one temporary, the
 * per-tetrahedron load sums (ntet doubles at the lowest order, ntet * dim P_{k-1} for the order-k
 * element, ntet = the cell tetrahedra of vem_get_quadrature), lives in a fixed device array of
 * 4 * 2^20 doubles (32 MiB) that the library holds on each device it runs on until the process
 * ends.  All handles on one device share that array, and every entry a call reads it writes first;
 * it keeps the last call's contents.  Two calls that overlap on one device (handles driven from
 * different host threads) race on it and must be serialised by the caller.  Errors as vem_set_rhs,
 * and VEM_ENOMEM (nothing changed) when the mesh needs more than the fixed array holds (about
 * 350,000 hexahedra at the lowest order): use vem_set_rhs there. */
vem_status vem_set_rhs_noalloc(vem_handle h, const double* f_qp, const double* pD_qp);

/* Select the boundary data: VEM_BC_PRESSURE (the default) or VEM_BC_FLUX, before or after
 * vem_discretize; a change clears the right-hand side.  With VEM_BC_FLUX the DOFs of the
 * boundary faces are prescribed: they hold identity rows and columns in K and A_gamma, B has no
 * column for them (so S neither), the right-hand side comes from vem_set_rhs_flux, Block-Schur's
 * inner solve takes the part of r_p orthogonal to the constant pressure (the kernel of S), and
 * vem_solve returns, of the pressures that solve the system, the one with zero mean
 * (sum_P |P| p_{P,0} = 0).  vem_set_rhs then fails with VEM_EINVAL. */
vem_status vem_set_boundary(vem_handle h, int kind);

/* Right-hand side with flux boundary data (Section 3, eq. mod_prob_eq): f_qp[n_qp_cell] as in
 * vem_set_rhs, and u_qp[3*n_qp_face] the flux field u at the boundary points of
 * vem_get_quadrature (structure of arrays: all x components, then y, then z; device).  The
 * prescribed DOFs are the face moments (1/|f|) int_f (u.n_f) m^f_b (eq. facePoly) with n_f the
 * face's global normal.  The system's right-hand side (b - K x_B on the free rows, x_B on the
 * prescribed ones, its pressure part projected off the constant pressure, which removes the
 * quadrature-level mismatch between int f and the boundary flux) depends on the coefficient and
 * is formed when it is used; vem_get_rhs returns it.  VEM_EINVAL unless the boundary data kind is
 * VEM_BC_FLUX. */
vem_status vem_set_rhs_flux(vem_handle h, const double* f_qp, const double* u_qp);

/* Solve the saddle system of eq. mod_prob_eqDisc, [M B^T; B 0][u; p] = [g; -F], by FGMRES with the
 * block preconditioner opts->precond (Section 5, eqs. block_schur and block_diag).  u[n_u], p[n_p]:
 * caller-owned device buffers receiving the flux and pressure unknowns (read as the initial guess
 * when opts->use_x0).  Blocks until the result is known.  Returns VEM_OK, VEM_NOT_CONVERGED (best
 * iterate written), or an error (VEM_EINVAL for bad options, VEM_ENAN, VEM_EHIP).  info may be
 * NULL. */
vem_status vem_solve(vem_handle h, const vem_solve_opts* opts, double* u, double* p, vem_solve_info* info);

/* Solve K x = rhs (K the matrix of eq. mod_prob_eqDisc) for a caller-supplied right-hand side
 * (device, n doubles) instead of the assembled [g; -F]; otherwise as vem_solve.  K is
 * symmetric (eq. mod_prob_eqDisc in the symmetric form above), so this is also
 * the adjoint solve K^T lambda = dJ/dx of a functional J of the solution
 * (same operator, same preconditioners).  Pressure boundary data only:
 * VEM_EINVAL with VEM_BC_FLUX, where K is singular and its prescribed rows fix
 * the boundary DOFs. */
vem_status vem_solve_rhs(vem_handle h, const vem_solve_opts* opts, const double* rhs, double* u, double* p,
                         vem_solve_info* info);

/* Per-cell derivative for the adjoint method (Section 4.3: M_P = nu_P M1_P
 * with nu piecewise constant): g[P] = nu_P lambda_P^T M1_P u_P, with u_P and
 * lambda_P the cell's oriented local flux DOFs of the device vectors u and
 * lam (n_u doubles each).  For nu = exp(-log K) and K x = b, a functional J
 * of x with K lambda = dJ/dx has dJ/d(log K_P) = g[P].  g: device, n_cells.
 * Pressure boundary data only: VEM_EINVAL with VEM_BC_FLUX (there the
 * prescribed boundary fluxes do not depend on K, and the formula would add
 * their terms). */
vem_status vem_coefficient_gradient(vem_handle h, const double* u, const double* lam, double* g);

/* y = K x for device vectors of length n (test hook for the saddle SpMV). */
vem_status vem_apply(vem_handle h, const double* x, double* y);

/* Copy a matrix out in CSR form to device buffers rowptr[rows+1], col[nnz],
 * val[nnz]; rows = n (VEM_MAT_K), n_p (VEM_MAT_SCHUR), n_u (VEM_MAT_REG),
 * n_face_dofs (VEM_MAT_REG_FACE, VEM_MAT_REG_SCHWARZ).  With col and val NULL only rowptr is
 * written (nnz = rowptr[rows]).  The two Schwarz matrices are built for the default gamma = h^2
 * if no Block-Reg solve has built them yet, else for the last solve's gamma. */
vem_status vem_export_csr(vem_handle h, int which, int32_t* rowptr, int32_t* col, double* val);

/* Copy the assembled right-hand side b = [g; -F] (device, n doubles). */
vem_status vem_get_rhs(vem_handle h, double* b);

/* Geometry export (device buffers, any may be NULL): face area[nf],
 * normal[nf*3], centroid[nf*3]; cell volume[nc], centroid[nc*3],
 * diameter[nc]. */
vem_status vem_get_geometry(vem_handle h, double* face_area, double* face_normal, double* face_centroid,
                            double* cell_volume, double* cell_centroid, double* cell_diam);

/* Hot kernels that vem_time_kernel can time. */
enum { VEM_KERNEL_SPMV = 0, VEM_KERNEL_CG_SCHUR = 1, VEM_KERNEL_CG_REG = 2, VEM_KERNEL_CG_SCHUR32 = 3,
       VEM_KERNEL_CG_REG32 = 4, VEM_KERNEL_CG_SCHUR32P = 5, VEM_KERNEL_CG_REG32P = 6,
       VEM_KERNEL_CG_REG_SCHWARZ = 7, VEM_KERNEL_CG_REG_SCHWARZ32 = 8, VEM_KERNEL_CHEB_SCHUR = 9,
       VEM_KERNEL_CHEB_SCHUR32 = 10 };

/* Measurement hook for benchmarks: time `reps` back-to-back launches of one
 * hot kernel with HIP events recorded on the handle's stream (the Chebyshev
 * products: each launch with start and stop events of its own, so that the
 * mean is the kernels' own time, without the dispatch gaps between launches).
 *   VEM_KERNEL_SPMV:     the saddle product y = K x;
 *   VEM_KERNEL_CG_SCHUR: one pipelined inner-CG iteration on S (Block-Schur);
 *   VEM_KERNEL_CG_REG:   one pipelined inner-CG iteration on M + B^T B / gamma;
 *   VEM_KERNEL_CG_SCHUR32, VEM_KERNEL_CG_REG32: one classical FP32 iteration (two
 *                        launches; VEM_MIXED with an inner cap above 64);
 *   VEM_KERNEL_CG_SCHUR32P, VEM_KERNEL_CG_REG32P: one pipelined FP32 iteration
 *                        (VEM_MIXED with an inner cap of 64 or less);
 *   VEM_KERNEL_CG_REG_SCHWARZ, VEM_KERNEL_CG_REG_SCHWARZ32: one iteration of Block-Reg's inner CG
 *                        with the edge-patch Schwarz preconditioner (two launches), FP64 / FP32;
 *   VEM_KERNEL_CHEB_SCHUR, VEM_KERNEL_CHEB_SCHUR32: one Chebyshev-Jacobi product on S (the
 *                        VEM_INNER_CHEBYSHEV form), FP64 / FP32.
 * avg_ms receives the mean duration of one launch; bytes (may be NULL) the
 * algorithmic bytes one launch moves (every matrix entry and every vector
 * element read or written once).  Uses the solver workspace; the results of
 * a previous vem_solve are not affected. */
vem_status vem_time_kernel(vem_handle h, int which, int reps, double* avg_ms, double* bytes);

const char* vem_status_string(vem_status st);
const char* vem_last_error(vem_handle h);

#ifdef __cplusplus
}
#endif

#endif /* VEM_H */
