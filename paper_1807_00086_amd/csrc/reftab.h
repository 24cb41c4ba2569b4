// Reference-element tables for the HDG local operators (host, FP64).
//
// Section 2.2: the volume spaces are P_k on the reference simplex mapped affinely to each
// element, the trace space is P_kF on the reference face mapped to each face.  All element
// matrices of the three physics are combinations of the tables below, scaled by
// per-element geometric factors (affine maps: constant Jacobian).
#pragma once
#include <cstdint>
#include <vector>

namespace hdg {

int dim_p(int k, int d);                        // dim P_k on the d-simplex

// Orthonormal PKD basis of P_k on the [0,1]-simplex of dimension d (1, 2 or 3), hierarchical
// by total degree.  val[N], grad[N*d] (grad may be null).
void pkd_eval(int d, int k, const double* xi, double* val, double* grad);

// Quadrature on the [0,1]-simplex: conical product of Gauss-Jacobi rules with q points per
// direction; exact for total degree 2q-1.
void simplex_quadrature(int d, int q, std::vector<double>& pts, std::vector<double>& wts);

// Number of vertex permutations of a face (2 for edges, 6 for triangles) and the p-th one.
int n_face_perms(int d);
void face_perm(int d, int p, int* perm);       // perm[0..d-1]

struct RefTables {
    int d = 0, k = 0, N = 0;
    int nf = 0;                                  // faces per element = d+1
    // Sr[r][i][j] = int phi_i d(phi_j)/d xi_r         (d x N x N)
    std::vector<double> Sr;
    // Mf[f][i][j] = int_{ref face} phi_i phi_j         ((d+1) x N x N), per unit ref-face measure
    std::vector<double> Mf;
    // Tsym[c][i][j]: c over the symmetric pairs (r,s), r<=s:  Sr[r] Sr[s]^T (+ transpose if r<s)
    std::vector<double> Tsym;
    // Tfull[r][s][i][j] = (Sr[r] Sr[s]^T)[i][j]   (d x d x N x N)
    std::vector<double> Tfull;
};

// Ef[kF][f][p][i][l] = int_{ref face} phi_i(xi_{f,p}(s)) psi_l(s) ds for face degree kF:
// the trace of volume function i on local face f paired with face basis function l, when the
// face parametrisation starts at local vertex perm_p(...) (see face_perm).
struct RefFaceTables {
    int d = 0, k = 0, kF = 0, N = 0, NF = 0, nperm = 0;
    std::vector<double> E;                       // (d+1) x nperm x N x NF
};

void build_ref_tables(int d, int k, RefTables& T);
void build_face_tables(int d, int k, int kF, RefFaceTables& E);


// Sorted local vertex list of local face f of a d-simplex (the d vertices other than f).
void local_face_vertices(int d, int f, int* lv);

}  // namespace hdg
