// Internal state of an HDG context (host + device buffers).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hdg.h"
#include "reftab.h"

namespace hdg {

constexpr int GEOM_STRIDE = 32;   // doubles per element geometry record
// 3D record: [0] |J|, [1..9] G = J^{-1} row-major (G[r][x] = d xi_r / d x_x),
//            [10..13] s_f = face measure / reference-face measure, [14..25] outward unit
//            normals n_f (4 x 3), [26..28] material (rho,c,-)|(rho,lambda,mu)|(eps,mu,sigma),
//            [29] stabilisation (tau or S)
// 2D record: [0] |J|, [1..4] G, [5..7] s_f, [8..13] normals (3 x 2), [26..29] as above
inline int geo_G(int) { return 1; }
inline int geo_s(int d) { return 1 + d * d; }
inline int geo_n(int d) { return 1 + d * d + (d + 1); }
constexpr int GEO_PAR = 26;
constexpr int GEO_STAB = 29;

struct DeviceTables {         // one polynomial degree (uniform meshes: face degree = k)
    int k = 0, N = 0, NF = 0;
    double *Sr = nullptr, *Mf = nullptr, *Tsym = nullptr, *Ef = nullptr;     // FP64
    double* Tfull = nullptr;
    float *Sr32 = nullptr, *Mf32 = nullptr, *Tsym32 = nullptr, *Ef32 = nullptr;
    float* Tfull32 = nullptr;
    // transposed FP64 copies (3D): SrT[r][j][i] = Sr[r][i][j], EfT[f][p][l][i] = Ef[f][p][i][l]
    double *SrT = nullptr, *EfT = nullptr;
};

struct Timings {
    float condense = 0, assemble = 0, solve = 0, recover = 0, refine_elem = 0, refine_solve = 0;
};

}  // namespace hdg

// workgroups of the reductions over the trace vectors (partial sums per workgroup and column)
constexpr int RED_MAX = 2048;
// doubles of the file-scope device scratch of hdg_trace_solve_static (64 MiB per GPU)
constexpr int64_t TRACE_STATIC_DOUBLES = (int64_t)8 << 20;

struct hdg_ctx {
    // configuration
    int dim = 0, physics = 0, precision = 0, nrhs = 1, k = 0;
    bool uniform = true;
    double stab_scale = 1.0;
    double krylov_tol = 1e-13, refine_tol = 1e-13, refine_inner_tol = 1e-6;
    int krylov_maxit = 2000, refine_maxit = 8;
    hipStream_t stream = nullptr;
    std::string err;

    // sizes
    int64_t n_elem = 0, n_vert = 0, n_faces = 0, n_bfaces = 0;
    int m_local = 0, m_trace = 0;
    int N = 0, NF = 0, n_loc = 0, n_tr = 0;   // per element (uniform degree)
    int64_t n_local_dofs = 0, n_trace_dofs = 0;
    int bs = 0;                                // trace block size per face = m_trace * NF
    int nslot = 0;                             // BSR blocks per face row = 1 + 2 d
    double K_sign = 1.0;                       // assemble sign * K so the system is SPD

    // host mesh data
    std::vector<double> xyz, par;
    std::vector<int64_t> ev;
    std::vector<int8_t> degree;
    std::vector<int32_t> elem_face;            // [ne][d+1]
    std::vector<int32_t> elem_perm;            // [ne][d+1]
    std::vector<int32_t> face_elem;            // [nf][2]
    std::vector<int32_t> face_lf;              // [nf][2]
    std::vector<int64_t> face_vert;            // [nf][d] sorted global ids
    std::vector<uint8_t> face_bnd;             // [nf] 0 interior, 1 Dirichlet, 2 Neumann
    int64_t n_neumann = 0;
    std::vector<double> geom;                  // [ne][GEOM_STRIDE]
    std::vector<double> frame;                 // [nf][6] Maxwell tangent frame (t1, t2)
    std::vector<int64_t> bface_list;           // boundary faces in face order
    std::vector<int32_t> bsr_cols_h;           // [nf][nslot]

    hdg::RefTables ref;
    hdg::RefFaceTables reff;

    // device mesh data
    double* d_geom = nullptr;
    int32_t* d_eface = nullptr;
    int32_t* d_eperm = nullptr;
    int32_t* d_face_elem = nullptr;
    int32_t* d_face_lf = nullptr;
    uint8_t* d_face_bnd = nullptr;
    int32_t* d_bsr_cols = nullptr;
    double* d_eframe = nullptr;    // [ne][d+1][6] face frames of each element's faces (Maxwell)
    void* d_xscratch = nullptr;    // per-workgroup condensation scratch when it exceeds LDS
    hdg::DeviceTables tab;

    // condensation outputs (precision-typed: double or float)
    void* d_Ke = nullptr;      // [ne][t][t]
    void* d_re = nullptr;      // [ne][t][r]
    void* d_Zt = nullptr;      // [ne][Ns][t]  rows of Z = A^{-1} B for the Schur block (the
                               // acoustic kernels of the fast path store it column-major, [ne][t][Ns])
    void* d_z = nullptr;       // [ne][n][r]
    void* d_LU = nullptr;      // [ne][Ns][Ns] factored Schur block (mixed precision; acoustic fast
                               // path: U = diag(d) L_u^T column-major, inverse pivots on the diagonal)
    int Ns = 0;                // size of the densely factored (Schur) block
    int ke_tile = 0;           // > 0: K_e holds only the entries whose row tile (of this many
                               // rows) is <= their column tile; the rest is read mirrored
    int s_row0 = 0;            // first local row of that block
    int* d_status = nullptr;   // device status word (0 ok, 1 singular pivot)

    // routing: the acoustic kernels of condense_acoustic.hip serve uniform degree with one
    // right-hand side; every other configuration goes through the block-structured kernels
    bool fast_ac = false;
    // cached factors (acoustic fast path): the condensation also keeps U of every element so
    // that hdg_condense_rhs can condense a new right-hand side with the same stage coefficient
    bool cache_factors = false;
    bool factors_cached = false;   // the last hdg_condense left Z_p, U and K assembled
    // variable polynomial degree (acoustic, 3D): degree classes, compact local offsets, per-face
    // sizes.  n_loc, N, Ns are then the strides of the largest class and NF, bs, n_tr those of
    // the face tables (degree 5); faces of lower degree are padded.
    bool vardeg = false;
    size_t xscratch_bytes = 0;
    std::vector<int64_t> loc_off_h;  // [ne + 1]
    int64_t* d_loc_off = nullptr;
    int8_t* d_efnf = nullptr;        // [ne][d+1] face space size of each local face
    int8_t* d_face_nf = nullptr;     // [nf] face space size of each face
    int8_t* d_edeg = nullptr;        // [ne] element degree
    int64_t cls_n[6] = {0, 0, 0, 0, 0, 0};
    int32_t* d_cls[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    hdg::DeviceTables tabk[6];       // tables of each element degree (face tables of degree 5)

    // global trace system (FP64)
    double* d_bsr = nullptr;   // [nf][nslot][bs][bs]
    float* d_bsr32 = nullptr;  // FP32 copy for the correction solves of the refinement (mixed
                               // precision, 1 or 32 right-hand sides, 3D)
    double* d_rhs = nullptr;   // [ntr][r]
    double* d_pinv = nullptr;  // [nf][bs][bs] inverse diagonal blocks
    double *d_cg_r = nullptr, *d_cg_z = nullptr, *d_cg_p = nullptr, *d_cg_q = nullptr;
    double* d_red = nullptr;   // reduction scratch: RED_MAX x 32 partial sums
    double* d_scal = nullptr;  // device scalars
    int red_blocks = 0;

    // stage / refinement buffers (FP64)
    double* d_f_saved = nullptr;     // [n_local_dofs][r]
    double* d_lbnd_saved = nullptr;  // [n_trace_dofs][r]
    double* d_su = nullptr;          // [n_local_dofs][r]
    double* d_slam = nullptr;        // [n_trace_dofs][r]
    double* d_du = nullptr;          // [n_local_dofs][r] correction
    double* d_dlam = nullptr;        // [n_trace_dofs][r] correction
    double* d_re64 = nullptr;        // [ne][t][r] FP64 correction trace right-hand side
    double* d_sq = nullptr;          // refinement norms: acoustic fast path [3][ne] (|du|, |u|, |s_p| per
                                     // element), otherwise [ne][r] (|s| per element and column)
    double* d_stage = nullptr;       // [3][n_local_dofs][r] DIRK stages
    double* d_ustar = nullptr;
    double* d_fstage = nullptr;
    double last_a = 0.0;
    bool condensed = false;
    bool z_consumed = false;         // mixed: z buffer reused by the refinement corrections
    int last_iters = 0, last_refine = 0;
    // relative FP64 residual per column of the final iterate of the last mixed-precision recover
    double last_resid[32] = {};
    bool has_resid = false;
    hdg::Timings tim;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;

    // launch schedules of the block-structured condensation (index: [FP32 | FP64][degree]);
    // -1: not chosen yet.  Autotuning times every built schedule of a class on its first
    // condensation; the table file keeps the choices across contexts.
    bool autotune = false;
    std::string tune_path, device_name;
    int8_t sched[2][6] = {{-1, -1, -1, -1, -1, -1}, {-1, -1, -1, -1, -1, -1}};
    float sched_ms[2][6][5] = {};   // per precision, degree, launch schedule
    size_t xs_off[6] = {0, 0, 0, 0, 0, 0};   // per-class offsets into d_xscratch (bytes)
    // one hipGraph per condensation of a mesh of variable degree: class launches on side
    // streams forked from and joined into side[0]
    bool use_graph = false;
    hipStream_t side[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    hipEvent_t ev_fork = nullptr, ev_in = nullptr, ev_out = nullptr;
    // trace CG: residual norms copied to pinned host memory while the next product runs
    double* h_rr = nullptr;   // [32], hipHostMalloc
    hipEvent_t ev_rr = nullptr;
    hipEvent_t ev_join[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    hipGraphExec_t gexec = nullptr;
    double g_a = 0.0;
    const double* g_f = nullptr;
    int g_sched = -1;

    // device-side CG (graph capture): launches of the iteration kernels read *cg_done and return
    // at once when it is set; null outside the captured solve
    const int* cg_done = nullptr;
    int* d_cgflags = nullptr;   // [3][2] per stage: done (1 converged, 2 non-finite), iterations
    // hdg_step as one graph (options.graph_step, FP64): the executable, the stream it was
    // captured on, and what it was captured for (a replay needs all of it unchanged)
    bool graph_step = false;
    hipGraphExec_t sgexec = nullptr;
    hipStream_t sg_stream = nullptr;
    struct StepKey {
        double dt = 0.0;
        int scheme = -1;
        const double *u = nullptr, *lambda = nullptr, *lam_bnd = nullptr, *src = nullptr;
        bool operator==(const StepKey& o) const {
            return dt == o.dt && scheme == o.scheme && u == o.u && lambda == o.lambda && lam_bnd == o.lam_bnd &&
                   src == o.src;
        }
    } sg_key;
    bool sg_reuse = false;      // captured with the factors of last_a kept (right-hand sides only)
    int sg_nit = 0;             // CG iterations per stage in the captured graph
    bool sg_replayed = false;   // the last hdg_step ran as a graph replay

    // multicolour block SSOR preconditioner of the trace CG (options.precond): face colours
    // (faces sharing an element differ), the faces of each colour, and work vectors
    int precond = 0;
    int ncolors = 0;
    std::vector<int64_t> color_off;   // [ncolors + 1] offsets into d_cfaces
    int32_t* d_cfaces = nullptr;      // [nf] faces grouped by colour (colour-order positions)
    int32_t* d_ssoff = nullptr;       // [2][nf + 1] first sweep block of each position: forward, backward
    int32_t* d_ssnb = nullptr;        // [ss_nblk] neighbour face of each sweep block
    int32_t* d_ssdst = nullptr;       // [nf][nslot - 1] sweep block of block-row slot s >= 1, or -1
    int64_t ss_nblk = 0;              // sweep blocks: the forward ones (lower colours) first
    double* d_ss = nullptr;           // [3][ntr]: t, u, y of the transformed CG (+ [n_faces][32] p.q partials with 32 rhs)
    double* d_ssA = nullptr;          // [ss_nblk][bs][bs] R_F^{-1} K_FG R_G^{-T} in sweep order
    double* d_rinv = nullptr;         // [nf][bs][bs] R_F^{-1}, D_F = R_F R_F^T (Cholesky)
    int64_t mat_version = 0;          // counts assemblies of the trace matrix
    int64_t ss_version = -1;          // assembly the scaled copy was built from
    int64_t pinv_version = -1;        // assembly the block-Jacobi inverses were built from
    int64_t bsr32_version = -1;       // assembly the FP32 copy of K was made from
    // device memory of the workspaces (options.dev_alloc / dev_free; null: hipMalloc / hipFree)
    void* (*dev_alloc)(void*, size_t) = nullptr;
    void (*dev_free)(void*, void*) = nullptr;
    void* alloc_user = nullptr;
};

namespace hdg {
// mesh.cpp
int build_mesh(hdg_ctx* c, const hdg_mesh_desc* m, const hdg_phys_desc* p);
// device memory through the context's allocator (hipMalloc when none is set); hipError_t as int
int dev_malloc(hdg_ctx* c, void** p, size_t bytes);
void dev_release(hdg_ctx* c, void* p);
// kernels (launchers, in .hip files); all return hipError_t as int
int launch_condense(hdg_ctx* c, double a, const double* f_loc, const double* lam_bnd);
int launch_assemble(hdg_ctx* c, const double* lam_bnd);
int launch_residual(hdg_ctx* c, double a, const double* u, const double* lam, const double* f,
                    const double* lam_bnd, double* su, double* slam);
// Acoustic recovery of (v, p) from the stored factors (FP64: the plain recovery; mixed
// precision: then, with resid = 1, the FP64 residual, the correction right-hand side and the
// element part of the trace residual; with resid = 2 the FP64 residual only: re64 = -t_e and
// nrm[2 ne + e] = |s_p|).  mode 1 starts from p = 0 with dlam = lam (the first recovery), mode 0
// applies the correction dlam, mode 2 none.  nrm: [3 ne] per-element |du|, |u|, |s_p| (|du| is
// not written by the check, resid = 2).
int launch_refine_acoustic(hdg_ctx* c, const double* lam, const double* dlam, int mode, int resid,
                           double* u, double* nrm);
// Right-hand-side condensation with the factors of the last condensation (acoustic fast path):
// r_e and z for a new f_loc; launch_assemble_rhs then assembles the trace right-hand side only.
int launch_condense_rhs_acoustic(hdg_ctx* c, double a, const double* f_loc);
int launch_assemble_rhs(hdg_ctx* c, const double* lam_bnd);
int launch_assemble_rhs64(hdg_ctx* c, const double* re64, const double* lam_bnd);
int launch_apply_mass(hdg_ctx* c, double a, const double* u, double* f);
int launch_block_inverse(hdg_ctx* c);
// lowp: products with the FP32 copy of the matrix (correction solves of the refinement, whose
// tolerance is far above FP32 rounding; the refinement's FP64 residual removes the difference)
int trace_cg(hdg_ctx* c, double* lambda, double tol, int* iters, double* relres, bool lowp = false);
// The same CG with a fixed number of iterations and the convergence test on the device (for
// graph capture): flags [2] = done, iterations; relres_dev = largest relative residual.
int trace_cg_device(hdg_ctx* c, double* x, double tol, int nit, int* flags, double* relres_dev);
int launch_zero_ints(hdg_ctx* c, int* p, int n);
// multicolour block SSOR (Eisenstat form) CG; returns HDG_OK / HDG_E_NOCONV / a HIP error
int trace_cg_ssor(hdg_ctx* c, double* x, double tol, int* iters, double* relres);
// the SSOR CG for graph capture (see trace_cg_device); its buffers come from trace_ssor_alloc,
// which must run before the capture
int trace_cg_ssor_device(hdg_ctx* c, double* x, double tol, int nit, int* flags, double* relres_dev);
int trace_ssor_alloc(hdg_ctx* c);
bool ssor_supported(const hdg_ctx* c);
int launch_bsr_f32(hdg_ctx* c);
// trace solve with the CG work vectors and reduction scratch in the library's static device
// array (no allocation); static_scratch_setup looks up the array's address on the current device
// once; trace_static_need is the number of doubles a context's solve needs
int static_scratch_setup();
int64_t trace_static_need(const hdg_ctx* c);
int trace_cg_static(hdg_ctx* c, double* lambda, int* iters, double* relres);

// Workgroups that stay resident on the whole device at once for `kernel` with `block` threads
// (at least 1): a grid of this size visits every element with one wave per element slot.
int resident_groups(const void* kernel, int block);
int launch_axpy(hdg_ctx* c, int64_t n, double alpha, const double* x, double* y);
int launch_lincomb(hdg_ctx* c, int64_t n, double a, const double* x, double b, const double* y,
                   double* out);
int launch_norm2(hdg_ctx* c, int64_t n, const double* x, double* host_out);
// sum of squares per column of a row-major [n][R] vector (R <= 32) to the host (synchronises);
// bnd_only: rows of the Dirichlet faces of a trace vector only (n = faces x bs)
int launch_col_sq(hdg_ctx* c, int64_t n, int R, const double* x, double* host_out, bool bnd_only = false);
// condense_general.hip (elastodynamics, Maxwell)
bool general_supported(int physics, int k, int kf, int nrhs);
int var_face_degree();   // face-table degree used on meshes of variable degree
int launch_condense_general(hdg_ctx* c, double a, const double* f_loc);
// autotune table (capi.cpp): read the entries of this context, write the tuned ones back
void read_tune_table(hdg_ctx* c);
void write_tune_table(const hdg_ctx* c);
int launch_recover_general(hdg_ctx* c, const double* lam, double* u);
// FP64 residual of the full stage system at (u, lam) and, unless `check`, the correction right-hand
// side (re64) and the element part of the correction (z buffer); with `check` only re64 = -t_e
// and nrm[e][q] = |s| of element e, column q.
int launch_refine_general(hdg_ctx* c, const double* u, const double* lam, bool check, double* nrm);
// Right-hand-side condensation with the factors kept by the last condensation (block-structured
// path, one right-hand side; the factor of the Schur block is kept with options.cache_factors in
// FP64 and always in mixed precision): z and r_e of f_loc
int launch_condense_rhs_general(hdg_ctx* c, const double* f_loc);
// recover_mrhs.hip (acoustic, 3D, 32 right-hand sides: matrix-core recovery and refinement)
bool mr_supported(const hdg_ctx* c);
int launch_recover_mr(hdg_ctx* c, const double* lam, double* u);
int launch_refine_mr(hdg_ctx* c, const double* u, const double* lam, bool check, double* nrm);
}  // namespace hdg
