// Mesh skeleton and per-element geometry (host).  Section 2.1: faces E_h = E_h^I U E_h^B; an
// interior face is shared by exactly two elements.  Faces are numbered in lexicographic
// order of their sorted global vertex ids; each element records, per local face, the global
// face id and which vertex permutation maps the face's sorted global order to its local
// vertex order (this selects the oriented trace table).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <sstream>

#include "internal.h"

namespace hdg {

namespace {
struct FaceRec {
    std::array<int64_t, 3> key;
    int32_t elem;
    int32_t lf;
    bool operator<(const FaceRec& o) const {
        if (key != o.key) return key < o.key;
        if (elem != o.elem) return elem < o.elem;
        return lf < o.lf;
    }
};

void cross3(const double* a, const double* b, double* c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
}  // namespace

int build_mesh(hdg_ctx* c, const hdg_mesh_desc* m, const hdg_phys_desc* p) {
    const int d = m->dim;
    const int nv = d + 1;
    const int64_t ne = m->n_elem;
    c->dim = d;
    c->n_elem = ne;
    c->n_vert = m->n_vert;
    c->xyz.assign(m->xyz, m->xyz + m->n_vert * d);
    c->ev.assign(m->elem_vert, m->elem_vert + ne * nv);
    for (int64_t i = 0; i < ne * nv; ++i)
        if (c->ev[i] < 0 || c->ev[i] >= m->n_vert) {
            c->err = "element vertex index out of range";
            return HDG_E_MESH;
        }

    // ---- faces
    std::vector<FaceRec> recs;
    recs.reserve(ne * nv);
    for (int64_t e = 0; e < ne; ++e)
        for (int f = 0; f < nv; ++f) {
            FaceRec r;
            r.key = {-1, -1, -1};
            int lv[3];
            local_face_vertices(d, f, lv);
            for (int q = 0; q < d; ++q) r.key[q] = c->ev[e * nv + lv[q]];
            std::sort(r.key.begin(), r.key.begin() + d);
            r.elem = (int32_t)e;
            r.lf = f;
            recs.push_back(r);
        }
    std::sort(recs.begin(), recs.end());
    c->elem_face.assign(ne * nv, -1);
    c->face_elem.clear();
    c->face_lf.clear();
    c->face_vert.clear();
    size_t i = 0;
    int64_t nf = 0;
    while (i < recs.size()) {
        size_t j = i;
        while (j < recs.size() && recs[j].key == recs[i].key) ++j;
        if (j - i > 2) {
            std::ostringstream os;
            os << "non-manifold face shared by " << (j - i) << " elements";
            c->err = os.str();
            return HDG_E_MESH;
        }
        for (int q = 0; q < d; ++q) c->face_vert.push_back(recs[i].key[q]);
        c->face_elem.push_back(recs[i].elem);
        c->face_lf.push_back(recs[i].lf);
        c->face_elem.push_back(j - i == 2 ? recs[i + 1].elem : -1);
        c->face_lf.push_back(j - i == 2 ? recs[i + 1].lf : -1);
        for (size_t q = i; q < j; ++q) c->elem_face[recs[q].elem * nv + recs[q].lf] = (int32_t)nf;
        ++nf;
        i = j;
    }
    c->n_faces = nf;
    // 0 interior, 1 Dirichlet, 2 Neumann
    c->face_bnd.assign(nf, 0);
    c->bface_list.clear();
    for (int64_t f = 0; f < nf; ++f)
        if (c->face_elem[2 * f + 1] < 0) {
            c->face_bnd[f] = 1;
            c->bface_list.push_back(f);
        }
    c->n_bfaces = (int64_t)c->bface_list.size();
    c->n_neumann = 0;
    if (m->bface_tag) {
        for (int64_t e = 0; e < ne; ++e)
            for (int f = 0; f < nv; ++f) {
                const int8_t t = m->bface_tag[e * nv + f];
                if (t == 0) continue;
                const int32_t F = c->elem_face[e * nv + f];
                if (t != 1) {
                    c->err = "bface_tag: 0 (Dirichlet) or 1 (Neumann) expected";
                    return HDG_E_MESH;
                }
                if (c->face_elem[2 * F + 1] >= 0) {
                    c->err = "bface_tag: Neumann tag on an interior face";
                    return HDG_E_MESH;
                }
                c->face_bnd[F] = 2;
                ++c->n_neumann;
            }
    }

    // ---- permutations of each element face
    c->elem_perm.assign(ne * nv, 0);
    const int np = n_face_perms(d);
    for (int64_t e = 0; e < ne; ++e)
        for (int f = 0; f < nv; ++f) {
            int lv[3];
            local_face_vertices(d, f, lv);
            int found = -1;
            for (int pp = 0; pp < np && found < 0; ++pp) {
                int perm[3];
                face_perm(d, pp, perm);
                bool inc = true;
                for (int q = 0; q + 1 < d; ++q)
                    if (!(c->ev[e * nv + lv[perm[q]]] < c->ev[e * nv + lv[perm[q + 1]]])) inc = false;
                if (inc) found = pp;
            }
            if (found < 0) {
                c->err = "degenerate face (repeated vertex)";
                return HDG_E_MESH;
            }
            c->elem_perm[e * nv + f] = found;
        }

    // ---- geometry
    c->geom.assign(ne * GEOM_STRIDE, 0.0);
    c->par.assign(ne * 3, 0.0);
    for (int64_t e = 0; e < ne; ++e) {
        double X[4][3] = {};
        for (int v = 0; v < nv; ++v)
            for (int r = 0; r < d; ++r) X[v][r] = c->xyz[c->ev[e * nv + v] * d + r];
        double J[3][3] = {}, G[3][3] = {};
        for (int r = 0; r < d; ++r)
            for (int s = 0; s < d; ++s) J[r][s] = X[s + 1][r] - X[0][r];
        double det;
        if (d == 2) {
            det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
            G[0][0] = J[1][1] / det;
            G[0][1] = -J[0][1] / det;
            G[1][0] = -J[1][0] / det;
            G[1][1] = J[0][0] / det;
        } else {
            det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                  J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                  J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
            // G = J^{-1}
            G[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
            G[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
            G[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
            G[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
            G[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
            G[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
            G[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
            G[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
            G[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
        }
        if (!(det > 0.0) || !std::isfinite(det)) {
            std::ostringstream os;
            os << "element " << e << " is inverted or degenerate (det J = " << det << ")";
            c->err = os.str();
            return HDG_E_MESH;
        }
        double* g = &c->geom[e * GEOM_STRIDE];
        g[0] = det;
        for (int r = 0; r < d; ++r)
            for (int s = 0; s < d; ++s) g[geo_G(d) + r * d + s] = G[r][s];
        for (int f = 0; f < nv; ++f) {
            int lv[3];
            local_face_vertices(d, f, lv);
            double nrm[3] = {}, meas;
            if (d == 2) {
                double t0 = X[lv[1]][0] - X[lv[0]][0], t1 = X[lv[1]][1] - X[lv[0]][1];
                meas = std::sqrt(t0 * t0 + t1 * t1);
                nrm[0] = t1 / meas;
                nrm[1] = -t0 / meas;
                g[geo_s(d) + f] = meas;
            } else {
                double a[3], b[3];
                for (int r = 0; r < 3; ++r) {
                    a[r] = X[lv[1]][r] - X[lv[0]][r];
                    b[r] = X[lv[2]][r] - X[lv[0]][r];
                }
                cross3(a, b, nrm);
                double nn = std::sqrt(nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2]);
                for (int r = 0; r < 3; ++r) nrm[r] /= nn;
                meas = 0.5 * nn;
                g[geo_s(d) + f] = 2.0 * meas;   // reference triangle has measure 1/2
            }
            // outward: away from the vertex opposite the face
            double dot = 0.0;
            for (int r = 0; r < d; ++r) dot += nrm[r] * (X[f][r] - X[lv[0]][r]);
            if (dot > 0)
                for (int r = 0; r < d; ++r) nrm[r] = -nrm[r];
            for (int r = 0; r < d; ++r) g[geo_n(d) + f * d + r] = nrm[r];
        }
        const double* pe = p->elem_par + e * 3;
        for (int q = 0; q < 3; ++q) {
            g[GEO_PAR + q] = pe[q];
            c->par[e * 3 + q] = pe[q];
        }
        double stab;
        if (p->physics == HDG_ACOUSTIC) {
            if (!(pe[0] > 0 && pe[1] > 0)) {
                c->err = "acoustic coefficients must be positive";
                return HDG_E_ARG;
            }
            stab = 1.0 / (pe[0] * pe[1]);
        } else if (p->physics == HDG_ELASTIC) {
            if (!(pe[0] > 0 && pe[2] > 0 && 3 * pe[1] + 2 * pe[2] > 0)) {
                c->err = "elastic coefficients out of range";
                return HDG_E_ARG;
            }
            stab = 2.0 * pe[0] * std::sqrt(pe[2] / pe[0]);
        } else {
            if (!(pe[0] > 0 && pe[1] > 0 && pe[2] >= 0)) {
                c->err = "Maxwell coefficients out of range";
                return HDG_E_ARG;
            }
            stab = 2.0;
        }
        g[GEO_STAB] = stab * c->stab_scale;
    }

    // ---- face frames (tangential traces)
    c->frame.assign(nf * 6, 0.0);
    if (d == 3)
        for (int64_t f = 0; f < nf; ++f) {
            const int64_t* fv = &c->face_vert[f * 3];
            double a[3], b[3], n[3], t2[3];
            for (int r = 0; r < 3; ++r) {
                a[r] = c->xyz[fv[1] * 3 + r] - c->xyz[fv[0] * 3 + r];
                b[r] = c->xyz[fv[2] * 3 + r] - c->xyz[fv[0] * 3 + r];
            }
            cross3(a, b, n);
            double nn = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
            double na = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
            for (int r = 0; r < 3; ++r) {
                n[r] /= nn;
                a[r] /= na;
            }
            cross3(n, a, t2);
            for (int r = 0; r < 3; ++r) {
                c->frame[f * 6 + r] = a[r];
                c->frame[f * 6 + 3 + r] = t2[r];
            }
        }

    // ---- BSR structure: slot 0 = diagonal, then for each neighbour side the other faces
    c->nslot = 1 + 2 * d;
    c->bsr_cols_h.assign(nf * c->nslot, -1);
    for (int64_t f = 0; f < nf; ++f) {
        c->bsr_cols_h[f * c->nslot] = (int32_t)f;
        for (int s = 0; s < 2; ++s) {
            int32_t e = c->face_elem[2 * f + s];
            if (e < 0) continue;
            int32_t lf = c->face_lf[2 * f + s];
            int m = 0;
            for (int q = 0; q < nv; ++q) {
                if (q == lf) continue;
                c->bsr_cols_h[f * c->nslot + 1 + s * d + m] = c->elem_face[e * nv + q];
                ++m;
            }
        }
    }
    return HDG_OK;
}

}  // namespace hdg
