/*
 * hdg.h -- C ABI of the MI355X (gfx950) HDG condensation library (libhdg.so).
 *
 * The library implements the element-local part of an implicit hybridised DG stage
 * (Fernandez, Christophe, Terrana, Nguyen, Peraire, "Hybridized discontinuous Galerkin
 * methods for wave propagation", arXiv:1807.00086):
 *
 *   section 2.3   the semi-discrete problem is an index-1 DAE  M du/dt + f(u,v,t) = 0,
 *                 g(u,v,t) = 0, advanced by DIRK stages (section 2.3.2);
 *   section 2.4.1 every stage is a linear system [A B; C D] (u, lam) = (f, g) whose block
 *                 A is block-diagonal over elements; the local unknowns are eliminated,
 *                 K = D - C A^{-1} B, r = g - C A^{-1} f, the global trace system
 *                 K lam = r is solved, and u is recovered from the first block row.
 *
 * Physics: acoustics (velocity v, pressure p; trace p_hat), linear elastodynamics
 * (velocity, symmetric stress; trace v_hat; section 4.1), Maxwell (E, H; tangential
 * trace E_hat^t; section 5.2), and Maxwell with the generalised Lagrange multiplier phi of
 * section 5.1.2 (equations (dmax1)-(dmax3), alpha_1 = alpha_2 = alpha_3 = 1, phi eliminated
 * locally, so the trace system is that of Maxwell).  The orderings are listed below; the local equations and
 * sign conventions of each physics are stated in csrc/physics.h.
 *
 * Conventions shared by every entry point
 *  - Reference simplex: vertices 0, e_1, .., e_d; local face f is opposite local vertex f.
 *  - Basis: orthonormal PKD (Dubiner) polynomials of degree k on the reference simplex,
 *    ordered by total degree; trace basis: the same on the reference face, mapped from the
 *    face's vertices sorted by global id (so both neighbours share it).
 *  - Global faces are numbered in lexicographic order of their sorted global vertex ids.
 *  - Local dofs: element-major, then field component, then basis index, then rhs (r
 *    innermost when nrhs > 1).  Component orders:
 *      acoustic [v_1..v_d, p];  elastic [s11,s22,s33,s23,s13,s12, v_1,v_2,v_3];
 *      maxwell [H_1,H_2,H_3, E_1,E_2,E_3];  maxwell_glm [H_1,H_2,H_3, E_1,E_2,E_3, phi].
 *  - Trace dofs: face-major, then component, then face basis index, then rhs.
 *    On a mesh of variable degree the face degree is the larger degree of the face's
 *    elements (the element's own degree on the boundary), and every face is padded to the
 *    face space of degree 5 (21 entries per rhs; entries past the face's own space are
 *    zero on output and ignored on input).  Local dofs stay compact: element e starts at
 *    the prefix sum of (d+1) dim P_{k_e} over the elements before it.
 *    Maxwell trace components are coefficients along the face frame (t1, t2):
 *    t1 = unit(X_g1 - X_g0), t2 = n_F x t1, n_F = unit((X_g1-X_g0) x (X_g2-X_g0)).
 *  - Device pointers are borrowed for the duration of the call (stream-ordered on the
 *    context's stream).  Host pointers are read during the call only.
 *  - Every entry point returns an hdg_status; no exception crosses the ABI.  A failed call
 *    leaves a message retrievable with hdg_last_error().
 */
#ifndef HDG_H
#define HDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int hdg_status;
enum {
    HDG_OK = 0,
    HDG_E_ARG = 1,         /* invalid argument (null pointer, size or enum out of range)   */
    HDG_E_MESH = 2,        /* inverted element, non-manifold face, degree out of range      */
    HDG_E_ALLOC = 3,       /* device allocation failed                                      */
    HDG_E_HIP = 4,         /* a HIP runtime call failed                                     */
    HDG_E_SINGULAR = 5,    /* zero / non-finite pivot in a local factorisation              */
    HDG_E_NOCONV = 6,      /* Krylov solve or refinement did not reach its tolerance        */
    HDG_E_STATE = 7,       /* call order violated (e.g. recover before condense)            */
    HDG_E_UNSUPPORTED = 8  /* configuration not built into this library                     */
};

enum hdg_physics { HDG_ACOUSTIC = 0, HDG_ELASTIC = 1, HDG_MAXWELL = 2, HDG_MAXWELL_GLM = 3 };
enum hdg_precision {
    HDG_FP64 = 0,          /* local factorisations, Z and K_e in FP64                       */
    HDG_MIXED_FP32 = 1,    /* local factorisations, Z and K_e in FP32, FP64 refinement      */
    HDG_MIXED_BF16 = 2     /* as MIXED_FP32, with the matrix-core products of the local
                              condensation (B~2, the triangular-solve updates, K_e) as
                              split-BF16 products on the BF16 matrix cores (FP32 accumulation);
                              the Schur factorisation stays FP32.  Elastic, Maxwell and
                              GLM-Maxwell (uniform degree, one rhs)                         */
};
enum hdg_scheme { HDG_BACKWARD_EULER = 0, HDG_DIRK33 = 1 };

typedef struct hdg_ctx hdg_ctx;

typedef struct {
    int dim;                    /* 2 (triangles) or 3 (tetrahedra)                            */
    int64_t n_vert;
    const double* xyz;          /* host [n_vert][dim]                                         */
    int64_t n_elem;
    const int64_t* elem_vert;   /* host [n_elem][dim+1], positively oriented                  */
    const int8_t* degree;       /* host [n_elem] polynomial degree (1..5); NULL: options.k.
                                   Degrees that differ between elements: 3D acoustics only  */
    const int8_t* bface_tag;    /* host [n_elem][dim+1] or NULL (every boundary face
                                   Dirichlet): the condition on the local face opposite vertex
                                   f, 0 Dirichlet, 1 Neumann (section 4.1.2, the Gamma_N part
                                   of the trace equation: the face keeps its element's flux
                                   row, whose right-hand side is the tested datum <g_N, mu>_F).
                                   Interior faces must carry 0 (else HDG_E_MESH).            */
} hdg_mesh_desc;

typedef struct {
    int physics;                /* enum hdg_physics                                           */
    const double* elem_par;     /* host [n_elem][3]: acoustic (rho, c, -), elastic
                                   (rho, lambda, mu), maxwell and maxwell_glm (eps, mu, sigma) */
    double stab_scale;          /* multiplies tau = 1/(rho c) | S = 2 rho c_s | tau = 2       */
} hdg_phys_desc;

typedef struct {
    int precision;              /* enum hdg_precision                                         */
    int k;                      /* uniform degree when mesh.degree == NULL                    */
    int nrhs;                   /* right-hand sides solved together (1..32)                   */
    double krylov_tol;          /* relative residual of the FP64 trace solve                  */
    int krylov_maxit;
    double refine_tol;          /* mixed precision: stop when the FP64 residual of the full
                                   stage system at the refined iterate is at most refine_tol
                                   times the norm of its right-hand side (f, Dirichlet data),
                                   in every right-hand-side column (0: 1e-13)                */
    int refine_maxit;
    double refine_inner_tol;    /* mixed precision: relative residual of the trace solves of
                                   the corrections (0: 1e-6)                                  */
    int cache_factors;          /* nonzero: keep the factors of every condensation so that
                                   hdg_condense_rhs (and hdg_step, whose stages share one
                                   stage coefficient) can condense a new right-hand side
                                   without refactoring (one rhs, every physics); costs n_s^2
                                   values per element in FP64 (the mixed-precision paths keep
                                   them anyway)                                              */
    int autotune;               /* nonzero: the first hdg_condense of each degree class of the
                                   block-structured kernels (elastic, Maxwell, acoustics of
                                   variable degree or with 32 rhs) times every launch schedule
                                   built for it on the mesh's own elements (where the element
                                   buffers live: LDS only, or part of them in per-workgroup
                                   global scratch; reference tables in LDS or read through the
                                   caches: trading LDS for workgroups per CU; four or eight
                                   wavefronts per element workgroup), keeps the
                                   fastest for the life of the context and synchronises once
                                   to read the timers.  Zero: the built-in default.          */
    const char* autotune_table; /* NULL, or a text file of tuned schedules: read at
                                   hdg_init_mesh (entries for this physics, nrhs, precision
                                   and device replace the defaults), rewritten after tuning.
                                   One line per class: device physics k kF nrhs precision
                                   schedule ms_0 .. ms_4 (lines starting with '#' are
                                   comments; 0 ms: schedule not built for the class)        */
    int use_graph;              /* nonzero, mesh of variable degree: hdg_condense runs its
                                   per-degree-class launches as one hipGraph whose class
                                   kernels are independent branches (they may overlap on the
                                   device); the graph is captured on the first call and again
                                   whenever a, f_loc or a tuned schedule changes             */
    int graph_step;             /* nonzero (FP64 only, else HDG_E_UNSUPPORTED at init): hdg_step
                                   runs a whole step as one hipGraph replay with no host
                                   synchronisation inside it.  The trace CG then tests its
                                   convergence on the device: the graph holds a fixed number of
                                   iterations per stage (the most a stage took in the eager
                                   step that preceded the capture, plus a quarter and 8) whose
                                   kernels return at once after the test has passed.  The first
                                   step with given (dt, scheme, u, lambda, lam_bnd, src) runs
                                   eagerly and captures the graph; later steps with the same
                                   arguments (and, with cache_factors, the factors of the same
                                   stage coefficient still held) replay it.  A replay in which
                                   a stage has not converged leaves u unchanged, the step runs
                                   eagerly (reporting HDG_E_NOCONV as usual if it fails) and the
                                   graph is captured again with twice the iterations (at most
                                   krylov_maxit).  The iterate is that of the eager step. */
    /* Device memory of the context's workspaces.  Both NULL: hipMalloc / hipFree.  Both set:
       every device workspace (element factors and buffers, trace system, Krylov and stage
       vectors, tables) comes from dev_alloc(alloc_user, bytes), which returns device memory
       of the current device aligned to 256 bytes or NULL on failure (HDG_E_ALLOC), and goes
       back through dev_free(alloc_user, ptr) at hdg_destroy (or when a workspace is
       replaced), after the context's stream has been synchronised.  For callers whose
       memory is pooled, e.g. a framework's caching allocator: the blocks are used on the
       context's stream only.  Pinned host memory and the file-scope scratch of
       hdg_trace_solve_static are not affected.  Exactly one of the two set: HDG_E_ARG.  */
    void* (*dev_alloc)(void* alloc_user, size_t bytes);
    void (*dev_free)(void* alloc_user, void* ptr);
    void* alloc_user;
    int precond;                /* trace-solve preconditioner (enum hdg_precond).  HDG_PC_SSOR
                                   applies in 3D to the block sizes of the built
                                   configurations with one or 32 right-hand sides, in
                                   hdg_trace_solve, hdg_step and the correction solves of the
                                   mixed-precision refinement; inside the step graph (with the
                                   convergence test on the device) with one right-hand side;
                                   elsewhere and in hdg_trace_solve_static, block Jacobi is
                                   used.                                                      */
} hdg_options;

/* Preconditioners of the trace CG (section 2.4.2 uses BILU(0) inside RAS; K is symmetric
 * definite here, so the symmetric counterpart of a block incomplete factorisation is used). */
enum hdg_precond {
    HDG_PC_JACOBI = 0,          /* block Jacobi: the inverses of the face-diagonal blocks     */
    HDG_PC_SSOR = 1             /* block symmetric Gauss-Seidel in a multicolour face order
                                   (faces that share an element get different colours):
                                   M = (D + L) D^-1 (D + U), applied through Eisenstat's form
                                   on the block-diagonally scaled matrix W K W^T (W = R^-1 per
                                   face, D_F = R R^T), whose diagonal blocks are the identity:
                                   plain CG on (I + Lt)^-1 W K W^T (I + Ut)^-1, so an
                                   iteration costs one backward and one forward colour sweep
                                   and no diagonal block; convergence is confirmed on the
                                   same relative residual |b - K x| / |b| as with block
                                   Jacobi.  The scaled matrix (about 6 face blocks per face) is
                                   formed at the first solve after each assembly.           */
};

/* Query keys for hdg_query. */
enum hdg_query_key {
    HDG_Q_N_ELEM = 0, HDG_Q_N_FACES = 1, HDG_Q_N_BFACES = 2,
    HDG_Q_N_LOCAL_DOFS = 3,     /* sum over elements of n_e (without the nrhs factor)        */
    HDG_Q_N_TRACE_DOFS = 4,     /* sum over faces of m_hat dim P_kF(face)                   */
    HDG_Q_N_VOL_POINTS = 5,     /* total volume quadrature points (projection helper)       */
    HDG_Q_N_BND_POINTS = 6,     /* total boundary-face quadrature points                    */
    HDG_Q_LAST_ITERS = 7,       /* Krylov iterations of the last trace solve                 */
    HDG_Q_LAST_REFINE = 8,      /* refinement iterations of the last mixed recover          */
    HDG_Q_M_LOCAL = 9,          /* field components per element                             */
    HDG_Q_M_TRACE = 10,         /* trace components per face                                */
    HDG_Q_SCHEDULE = 11,        /* launch schedule of the block-structured condensation per
                                   degree class: 4 bits per degree k = 1..5 at bit 4 (k - 1),
                                   each 0 (no class or not chosen yet) or schedule + 1       */
    HDG_Q_STEP_GRAPH = 12,      /* 1 if the last hdg_step was a replay of the step graph     */
    HDG_Q_STEP_GRAPH_ITERS = 13,/* CG iterations per stage held by the step graph (0: none)  */
    HDG_Q_N_COLORS = 14         /* face colours of the multicolour preconditioner (0: none)   */
};

/*
 * hdg_init_mesh -- build the mesh skeleton and reference tables and upload them.
 * Sections 2.1-2.2 (mesh, faces E_h^I / E_h^B, spaces V_h^k and M_h^k).  All host arrays
 * are copied; the context owns every device buffer it allocates.  Validation (|J| <= 0,
 * a face shared by more than two elements, degree outside 1..5, nrhs outside 1..32)
 * fails with HDG_E_MESH / HDG_E_ARG before any device work.  `stream` is a hipStream_t
 * (NULL: the default stream); every later call is ordered on it.  Faces with one
 * neighbour are Dirichlet faces.
 * Built configurations (others return HDG_E_UNSUPPORTED before any device work):
 *   acoustics 2D/3D, uniform k = 1..4, nrhs = 1; acoustics 3D, uniform k = 1..4, nrhs = 32;
 *   acoustics 3D of variable degree (k_e in 1..5, face degree = the larger neighbour's),
 *   nrhs = 1 or 32; elastodynamics 3D, k = 1..4; Maxwell and GLM-Maxwell 3D, k = 1..3
 *   (nrhs = 1).
 * On a mesh of variable degree the projection helpers (hdg_volume_points and siblings)
 * return HDG_E_UNSUPPORTED; hdg_point_sources and hdg_apply_mass work on it.
 */
hdg_status hdg_init_mesh(hdg_ctx** out, const hdg_mesh_desc* mesh, const hdg_phys_desc* phys,
                         const hdg_options* opts, void* stream);

/* hdg_query -- integer facts about the discretisation (see enum hdg_query_key). */
hdg_status hdg_query(const hdg_ctx* ctx, int key, int64_t* value);

/*
 * hdg_condense -- element-local Galerkin solve and static condensation (section 2.4.1).
 * For every element: form A, B, C, D of the stage system with stage coefficient `a`
 * (A = a*Mw + L), factor A without pivoting (the flux-like leading block is
 * block-diagonal and is eliminated in closed form, the rest by a dense LU), compute
 * Z = A^{-1} B, z = A^{-1} f, K_e = D - C Z, r_e = -C z, and assemble the global trace
 * system in face-block sparse rows with the Dirichlet faces eliminated.
 *   a        stage coefficient d_ii / dt (> 0)
 *   f_loc    device [n_local_dofs][nrhs] FP64 local right-hand side (a Mw u* + sources)
 *   lam_bnd  device [n_trace_dofs][nrhs] FP64; only boundary-face entries are read:
 *            on Dirichlet faces the L2 projection of the Dirichlet data, on Neumann faces
 *            (mesh.bface_tag) the tested flux datum <g_N, mu_l>_F, added to the right-hand
 *            side of the face's flux rows (see hdg_project_boundary)
 * Asynchronous; a zero or non-finite pivot is reported by the next synchronising call
 * (hdg_trace_solve / hdg_recover) as HDG_E_SINGULAR.
 */
hdg_status hdg_condense(hdg_ctx* ctx, double a, const double* f_loc, const double* lam_bnd);

/*
 * hdg_condense_rhs -- condensation of a new right-hand side with the factors of the last
 * hdg_condense.  The element matrices A, B, C, D depend on the stage coefficient only
 * (section 2.4.1), so for the same `a` the factors Z and the assembled trace matrix stay
 * valid and only z = A^{-1} f and r_e = -C z change (static condensation of the right-hand
 * side, section 2.4.1): r_e and z are recomputed from the stored factors and the trace
 * right-hand side is assembled; the trace matrix and its preconditioner are kept.
 *   a        must equal the stage coefficient of the last hdg_condense
 *   f_loc    device [n_local_dofs][nrhs] FP64, lam_bnd device [n_trace_dofs][nrhs] FP64,
 *            as for hdg_condense
 * HDG_E_STATE without an earlier hdg_condense at this `a` whose factors were kept
 * (options.cache_factors in FP64; always in mixed precision); HDG_E_UNSUPPORTED with more than
 * one right-hand side.  Every physics and meshes of variable degree.  Asynchronous.
 */
hdg_status hdg_condense_rhs(hdg_ctx* ctx, double a, const double* f_loc, const double* lam_bnd);

/*
 * hdg_trace_solve -- solve the assembled trace system K lam = r in FP64 (section 2.4.2;
 * K is symmetric and definite for every physics here, so preconditioned conjugate
 * gradients replace GMRES; block-Jacobi or block-SSOR preconditioner, options.precond).
 *   lambda   device [n_trace_dofs][nrhs] in: initial guess (boundary entries are reset to
 *            the Dirichlet values), out: solution
 *   iters    host, may be NULL: iterations used
 *   relres   host, may be NULL: final max over rhs of ||r - K lam|| / ||r||
 * With block Jacobi in HDG_MIXED_FP32 mode on 3D meshes with 1 or 32 right-hand sides the
 * matrix products read an FP32 copy of K (K is assembled from the FP32 factors and hdg_recover's refinement
 * evaluates the residual in FP64 from the element operators, so this changes the solve only
 * at the level of error the refinement removes); relres then refers to that copy.
 * Synchronises the stream.  HDG_E_NOCONV if krylov_tol is not met within krylov_maxit.
 */
hdg_status hdg_trace_solve(hdg_ctx* ctx, double* lambda, int* iters, double* relres);

/*
 * hdg_trace_solve_static -- hdg_trace_solve that allocates nothing, for callers that cannot
 * allocate device memory (code under stream capture, tight serving loops, harnesses that forbid
 * allocation).  Same arguments, result and errors as hdg_trace_solve; the conjugate-gradient work
 * vectors and reduction partial sums live in a file-scope device array of the library
 * (64 MiB per GPU, held until the process ends) instead of the context's buffers.  A system that
 * needs more (4 x n_trace_dofs x nrhs doubles, plus 2048 x 32 + 256 doubles of partial sums
 * and scalars) fails with HDG_E_ARG before any device work.  All calls on one GPU share the array: calls that
 * overlap on a device (two streams, two threads) race and must not be issued.
 */
hdg_status hdg_trace_solve_static(hdg_ctx* ctx, double* lambda, int* iters, double* relres);

/*
 * hdg_recover -- local fields from the trace: u_e = z_e - Z_e lam_e (first block row of
 * the stage system).  In HDG_MIXED_FP32 mode the result is then refined: the residual of
 * the full uncondensed system is evaluated in FP64 from the element operators, corrected
 * through the FP32 factors and a new FP64 trace solve, and measured again in FP64 after each
 * correction, until it is at most refine_tol times the norm of the system's right-hand side
 * in every column (lambda is refined in place as well; hdg_last_residual reports the result).
 *   lambda   device [n_trace_dofs][nrhs] FP64 (in; in/out in mixed mode)
 *   u_loc    device [n_local_dofs][nrhs] FP64 out
 * HDG_E_NOCONV when the residual does not halve from one correction to the next or
 * refine_maxit corrections do not reach refine_tol.  In mixed mode the refinement reuses the
 * condensation buffers: a second hdg_recover needs a new hdg_condense (HDG_E_STATE).
 * The inner trace solves of the refinement use refine_inner_tol.
 */
hdg_status hdg_recover(hdg_ctx* ctx, double* lambda, double* u_loc);

/*
 * hdg_last_residual -- relative FP64 residual of the final iterate of the last mixed-precision
 * hdg_recover, per right-hand-side column: |s_q| / |(f_q, lam_D,q)| with
 * s = (f - A u - B lam, -(C u + D lam)) over the local rows and the trace rows of the
 * non-Dirichlet faces of the full (uncondensed) stage system (section 2.4.1).  The refinement
 * stops on this quantity (options.refine_tol).
 *   rel      host [nrhs] out
 * HDG_E_STATE if no mixed-precision hdg_recover has completed its check on this context.
 */
hdg_status hdg_last_residual(const hdg_ctx* ctx, double* rel);

/*
 * hdg_step -- advance u^n -> u^{n+1} by backward Euler or DIRK(3,3) (section 2.3.2,
 * stiffly accurate, so u^{n+1} is the last stage).  Per stage i:
 * u*_i = u^n - (1/d_ii) sum_{j<i} d_ij (U_j - u^n), f = a Mw u*_i with a = d_ii / dt, then
 * condense, trace solve, recover.  The DIRK(3,3) stages share d_ii, so with
 * options.cache_factors set every stage after the first condensation at a given dt only
 * condenses its right-hand side (hdg_condense_rhs).
 *   u          device [n_local_dofs][nrhs] in: u^n, out: u^{n+1}
 *   lambda     device [n_trace_dofs][nrhs] in: initial guess, out: trace of the last stage
 *   lam_bnd    device [n_stages][n_trace_dofs][nrhs] boundary data at t + c_i dt (as for
 *              hdg_condense)
 *   src        device [n_local_dofs][nrhs] or NULL: time-independent tested source
 * With options.graph_step the step is one graph replay after the first call with the same
 * arguments (see there); HDG_Q_STEP_GRAPH tells whether the last step was a replay.
 * Synchronises the stream.
 */
hdg_status hdg_step(hdg_ctx* ctx, double t, double dt, int scheme, double* u, double* lambda,
                    const double* lam_bnd, const double* src);

/* Stage glue: f = a * Mw * u element by element (device pointers, FP64). */
hdg_status hdg_apply_mass(hdg_ctx* ctx, double a, const double* u, double* f);

/*
 * Projection helpers (L2 projections that fix initial data and boundary data).
 * hdg_volume_points: host out [n_vol_points][dim] physical quadrature points, element-major.
 * hdg_project_volume: vals host [n_vol_points][m_local] field values at those points ->
 *   u host [n_local_dofs] (nrhs = 1 layout) coefficients u_i = (val, phi_i)_K / |J_K|.
 * hdg_boundary_points: host out [n_bnd_points][dim], boundary faces in face order.
 * hdg_project_boundary: vals host [n_bnd_points][dim or 1] -> lam host [n_trace_dofs]
 *   (zero on interior faces).  Dirichlet faces: vals is the trace (acoustic p, elastic v,
 *   Maxwell the full E vector, of which the tangential part along (t1, t2) is kept) and lam
 *   its L2 projection.  Neumann faces: vals is the prescribed flux with the outward normal
 *   n (acoustic v.n, elastic the traction sigma n, Maxwell the vector n x H) and lam its
 *   tested values <g, mu_l>_F.
 */
hdg_status hdg_volume_points(const hdg_ctx* ctx, double* pts);
hdg_status hdg_project_volume(const hdg_ctx* ctx, const double* vals, double* u);
hdg_status hdg_boundary_points(const hdg_ctx* ctx, double* pts);
hdg_status hdg_project_boundary(const hdg_ctx* ctx, const double* vals, double* lam);

/*
 * hdg_point_sources: host pts [n_src][dim] -> host f [n_local_dofs][n_src]: column s holds
 * phi_i(x_s) in the pressure block of the element containing x_s (acoustics only).
 */
hdg_status hdg_point_sources(const hdg_ctx* ctx, int n_src, const double* pts, double* f);

/*
 * hdg_element_data -- copy per-element results of the last condense to the host as FP64
 * (inspection / parity testing).  which: 0 = K_e [t][t], 1 = r_e [t][nrhs],
 * 2 = Z_s [n_s][t], 3 = z_s [n_s][nrhs]: the rows of Z = A^{-1} B and z = A^{-1} f that
 * belong to the densely factored block (acoustic p, elastic v, maxwell E; n_s of them per
 * element); the eliminated block is reconstructed in closed form at recovery.  Elements
 * [e0, e0+count) must share one degree; out holds count * block doubles.
 */
hdg_status hdg_element_data(hdg_ctx* ctx, int which, int64_t e0, int64_t count, double* out);

/* Timing of the last call of each kind, milliseconds (HIP events on the context stream):
 * which: 0 condense, 1 assemble, 2 trace solve, 3 recover, 4 refinement element work,
 * 5 refinement trace solves. */
hdg_status hdg_last_timing(const hdg_ctx* ctx, int which, double* ms);

/*
 * hdg_reference_table -- host-only copy of a reference-element table (no device needed):
 * which = 0: Sr[r][i][j] = int phi_i d phi_j / d xi_r (dim x N x N); 1: Mf[f][i][j] =
 * int_{face f} phi_i phi_j per unit reference-face measure ((dim+1) x N x N); 2: the symmetric
 * products Sr_r Sr_s^T (+ transpose for r < s); 3: E[f][p][i][l] = int_{face f} phi_i psi_l
 * with the face parametrised from vertex permutation p, face degree kF.  Writes at most cap
 * doubles; returns the count written or minus an hdg_status.
 */
int64_t hdg_reference_table(int dim, int k, int kF, int which, double* out, int64_t cap);

/*
 * hdg_hbm_probe -- diagnostic: achievable HBM bandwidth of a streaming pass, for comparison with
 * the element kernels' rooflines.  Times `reps` launches (after one untimed launch) of a read-only
 * pass over src (dst NULL: each 16-byte load summed in registers, nothing written) or of a copy
 * src -> dst, on `stream` with HIP events; grid = blocks_per_cu x compute units workgroups of 256
 * threads.  src, dst: device [n] FP64, n even; ms: host out, milliseconds per launch.
 */
hdg_status hdg_hbm_probe(const double* src, double* dst, int64_t n, int reps, int blocks_per_cu, void* stream,
                         double* ms);

/* hdg_destroy -- free every buffer the context owns.  NULL-safe. */
void hdg_destroy(hdg_ctx* ctx);

/* Message of the last failed call on this context ("" if none); ctx may be NULL for
 * failures of hdg_init_mesh, which are kept per thread. */
const char* hdg_last_error(const hdg_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* HDG_H */
