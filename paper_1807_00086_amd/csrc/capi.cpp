// C ABI entry points (host).  Argument validation, device buffers, call ordering and the
// FP64 refinement / time-stepping loops; every arithmetic step on the element and trace data
// runs in the HIP kernels of condense_*.hip, trace.hip and stage.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <unistd.h>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "internal.h"

namespace hdg {
int launch_condense_acoustic(hdg_ctx* c, double a, const double* f_loc);
int launch_condense_general(hdg_ctx* c, double a, const double* f_loc);

int dev_malloc(hdg_ctx* c, void** p, size_t bytes) {
    if (!c->dev_alloc) return (int)hipMalloc(p, bytes);
    void* q = c->dev_alloc(c->alloc_user, bytes);
    if (!q) {
        *p = nullptr;
        return (int)hipErrorOutOfMemory;
    }
    if (reinterpret_cast<uintptr_t>(q) % 256 != 0) {   // the kernels' vector loads assume it
        c->dev_free(c->alloc_user, q);
        *p = nullptr;
        return (int)hipErrorInvalidValue;
    }
    *p = q;
    return 0;
}

void dev_release(hdg_ctx* c, void* p) {
    if (!p) return;
    if (c->dev_free) c->dev_free(c->alloc_user, p);
    else (void)hipFree(p);
}

// Autotune table: one line per tuned class, "device physics k kF nrhs precision schedule ms_0
// ms_1 ms_2 ms_3 ms_4" (0: schedule not built for the class); '#' starts a comment line.
namespace {
bool tune_key_matches(const hdg_ctx* c, const std::string& dev, int phys, int k, int kf, int nrhs, int prec) {
    const int kf_c = c->vardeg ? var_face_degree() : k;
    const bool has = c->vardeg ? (k >= 1 && k <= 5 && c->cls_n[k] > 0) : k == c->k;
    return has && dev == c->device_name && phys == c->physics && kf == kf_c && nrhs == c->nrhs && prec == c->precision;
}
}  // namespace

void read_tune_table(hdg_ctx* c) {
    FILE* fp = std::fopen(c->tune_path.c_str(), "r");
    if (!fp) return;
    char line[512];
    const int pi = c->precision == HDG_FP64 ? 1 : 0;
    while (std::fgets(line, sizeof line, fp)) {
        if (line[0] == '#') continue;
        char dev[128];
        int phys, k, kf, nrhs, prec, sch;
        if (std::sscanf(line, "%127s %d %d %d %d %d %d", dev, &phys, &k, &kf, &nrhs, &prec, &sch) != 7) continue;
        if (sch < 0 || sch > 4 || !tune_key_matches(c, dev, phys, k, kf, nrhs, prec)) continue;
        c->sched[pi][k] = (int8_t)sch;
    }
    std::fclose(fp);
}

void write_tune_table(const hdg_ctx* c) {
    // only classes timed by this context are (re)written; other lines are kept as they are
    const int pi = c->precision == HDG_FP64 ? 1 : 0;
    auto timed = [&](int k) { return k >= 1 && k <= 5 && c->sched[pi][k] >= 0 && c->sched_ms[pi][k][0] > 0; };
    std::vector<std::string> keep;
    if (FILE* fp = std::fopen(c->tune_path.c_str(), "r")) {
        char line[512];
        while (std::fgets(line, sizeof line, fp)) {
            char dev[128];
            int phys, k, kf, nrhs, prec, sch;
            if (line[0] != '#' && std::sscanf(line, "%127s %d %d %d %d %d %d", dev, &phys, &k, &kf, &nrhs, &prec, &sch) == 7 &&
                tune_key_matches(c, dev, phys, k, kf, nrhs, prec) && timed(k))
                continue;   // replaced below
            keep.emplace_back(line);
        }
        std::fclose(fp);
    }
    // written beside the table under a per-process name, then renamed over it (the rename is
    // atomic, so a reader sees either the old or the new table; concurrent writers: last wins)
    const std::string tmp = c->tune_path + ".tmp" + std::to_string((long)getpid());
    FILE* fp = std::fopen(tmp.c_str(), "w");
    if (!fp) return;
    if (keep.empty())
        std::fprintf(fp, "# device physics k kF nrhs precision schedule ms_0 ms_1 ms_2 ms_3 ms_4 (0: not built)\n");
    for (const auto& l : keep) std::fputs(l.c_str(), fp);
    for (int k = 1; k <= 5; ++k) {
        if (!timed(k) || !tune_key_matches(c, c->device_name, c->physics, k, c->vardeg ? var_face_degree() : k,
                                                     c->nrhs, c->precision))
            continue;
        std::fprintf(fp, "%s %d %d %d %d %d %d %.4f %.4f %.4f %.4f %.4f\n", c->device_name.c_str(), c->physics, k,
                     c->vardeg ? var_face_degree() : k, c->nrhs, c->precision, c->sched[pi][k], c->sched_ms[pi][k][0],
                     c->sched_ms[pi][k][1], c->sched_ms[pi][k][2], c->sched_ms[pi][k][3], c->sched_ms[pi][k][4]);
    }
    std::fclose(fp);
    std::rename(tmp.c_str(), c->tune_path.c_str());
}
}  // namespace hdg

using namespace hdg;

namespace {

thread_local std::string g_init_err;

int fail(hdg_ctx* c, int code, const std::string& msg) {
    if (c)
        c->err = msg;
    else
        g_init_err = msg;
    return code;
}

#define HIPCHK(call)                                                                          \
    do {                                                                                      \
        hipError_t _e = (call);                                                               \
        if (_e != hipSuccess) return fail(c, HDG_E_HIP, std::string(#call ": ") + hipGetErrorString(_e)); \
    } while (0)

template <typename T>
int dalloc(hdg_ctx* c, T** p, size_t count) {
    if (count == 0) count = 1;
    hipError_t e = (hipError_t)dev_malloc(c, (void**)p, count * sizeof(T));
    if (e != hipSuccess) {
        std::ostringstream os;
        os << "device allocation of " << count * sizeof(T) << " bytes failed: " << hipGetErrorString(e);
        return fail(c, HDG_E_ALLOC, os.str());
    }
    return HDG_OK;
}

template <typename T>
int upload(hdg_ctx* c, T** p, const std::vector<T>& h) {
    int s = dalloc(c, p, h.size());
    if (s) return s;
    HIPCHK(hipMemcpy(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    return HDG_OK;
}

int upload_f32(hdg_ctx* c, float** p, const std::vector<double>& h) {
    std::vector<float> f(h.begin(), h.end());
    return upload(c, p, f);
}

// transposed FP64 copies of Sr and of the oriented face tables (3D)
int upload_transposed(hdg_ctx* c, DeviceTables& t, const RefTables& ref, const RefFaceTables& ef) {
    if (ref.d != 3) return HDG_OK;
    const int N = ref.N, NF = ef.NF, P = ef.nperm;
    std::vector<double> st(ref.Sr.size()), et(ef.E.size());
    for (int r = 0; r < 3; ++r)
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j) st[((size_t)r * N + j) * N + i] = ref.Sr[((size_t)r * N + i) * N + j];
    for (int fp = 0; fp < 4 * P; ++fp)
        for (int i = 0; i < N; ++i)
            for (int l = 0; l < NF; ++l) et[((size_t)fp * NF + l) * N + i] = ef.E[((size_t)fp * N + i) * NF + l];
    int s = HDG_OK;
    if ((s = upload(c, &t.SrT, st)) || (s = upload(c, &t.EfT, et))) return s;
    return HDG_OK;
}

// FP64 and FP32 copies of the reference tables of one degree
int upload_tables(hdg_ctx* c, DeviceTables& t, const RefTables& ref, const RefFaceTables& ef) {
    int s = upload_transposed(c, t, ref, ef);
    if (s) return s;
    if ((s = upload(c, &t.Sr, ref.Sr)) || (s = upload(c, &t.Mf, ref.Mf)) || (s = upload(c, &t.Tsym, ref.Tsym)) ||
        (s = upload(c, &t.Ef, ef.E)) || (s = upload(c, &t.Tfull, ref.Tfull)) || (s = upload_f32(c, &t.Sr32, ref.Sr)) ||
        (s = upload_f32(c, &t.Mf32, ref.Mf)) || (s = upload_f32(c, &t.Tsym32, ref.Tsym)) ||
        (s = upload_f32(c, &t.Ef32, ef.E)) || (s = upload_f32(c, &t.Tfull32, ref.Tfull)))
        return s;
    return HDG_OK;
}

void dfree(hdg_ctx* c, void* p) { dev_release(c, p); }

struct EventTimer {
    hdg_ctx* c;
    float* out;
    explicit EventTimer(hdg_ctx* cc, float* o) : c(cc), out(o) { (void)hipEventRecord(c->ev0, c->stream); }
    ~EventTimer() {
        (void)hipEventRecord(c->ev1, c->stream);
        if (hipEventSynchronize(c->ev1) == hipSuccess) (void)hipEventElapsedTime(out, c->ev0, c->ev1);
    }
};

int check_status(hdg_ctx* c) {
    int h = 0;
    HIPCHK(hipMemcpyAsync(&h, c->d_status, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (h & 1) return fail(c, HDG_E_SINGULAR, "zero or non-finite pivot in a local factorisation");
    return HDG_OK;
}

bool supported(hdg_ctx* c) {
    // split-BF16 products: the block-structured kernels of elastic and (GLM-)Maxwell only
    if (c->precision == HDG_MIXED_BF16 && (c->physics == HDG_ACOUSTIC || c->vardeg || c->nrhs != 1)) return false;
    if (c->vardeg) {
        for (int k = 1; k <= 5; ++k)
            if (c->cls_n[k] && !general_supported(HDG_ACOUSTIC, k, var_face_degree(), c->nrhs)) return false;
        return true;
    }
    if (c->fast_ac) return c->k >= 1 && c->k <= 4;
    return c->dim == 3 && general_supported(c->physics, c->k, c->k, c->nrhs);
}

int launch_recover_any(hdg_ctx* c, const double* lam, double* u) {
    return c->fast_ac ? launch_refine_acoustic(c, lam, lam, 1, 0, u, nullptr) : launch_recover_general(c, lam, u);
}


}  // namespace

extern "C" {

const char* hdg_last_error(const hdg_ctx* ctx) { return ctx ? ctx->err.c_str() : g_init_err.c_str(); }

hdg_status hdg_init_mesh(hdg_ctx** out, const hdg_mesh_desc* m, const hdg_phys_desc* p, const hdg_options* o,
                         void* stream) {
    g_init_err.clear();
    hdg_ctx* c = nullptr;
    if (!out || !m || !p || !o) return fail(nullptr, HDG_E_ARG, "null argument");
    *out = nullptr;
    if (m->dim != 2 && m->dim != 3) return fail(nullptr, HDG_E_ARG, "dim must be 2 or 3");
    if (!m->xyz || !m->elem_vert || m->n_elem <= 0 || m->n_vert <= 0)
        return fail(nullptr, HDG_E_ARG, "empty mesh or null mesh arrays");
    if (m->n_elem >= (int64_t)1 << 31) return fail(nullptr, HDG_E_ARG, "too many elements");
    if (p->physics < 0 || p->physics > 3) return fail(nullptr, HDG_E_ARG, "unknown physics");
    if (p->physics != HDG_ACOUSTIC && m->dim != 3) return fail(nullptr, HDG_E_ARG, "elastic/maxwell need dim 3");
    if (!p->elem_par) return fail(nullptr, HDG_E_ARG, "null elem_par");
    if (o->precision != HDG_FP64 && o->precision != HDG_MIXED_FP32 && o->precision != HDG_MIXED_BF16)
        return fail(nullptr, HDG_E_ARG, "unknown precision");
    if (o->nrhs < 1 || o->nrhs > 32) return fail(nullptr, HDG_E_ARG, "nrhs must be in 1..32");
    if (!(p->stab_scale > 0)) return fail(nullptr, HDG_E_ARG, "stab_scale must be positive");
    int kk = o->k;
    bool uniform = true;
    if (m->degree) {
        kk = m->degree[0];
        for (int64_t e = 0; e < m->n_elem; ++e) {
            if (m->degree[e] < 1 || m->degree[e] > 5) return fail(nullptr, HDG_E_MESH, "degree outside 1..5");
            if (m->degree[e] != kk) uniform = false;
        }
    }
    if (kk < 1 || kk > 5) return fail(nullptr, HDG_E_MESH, "degree outside 1..5");
    c = new (std::nothrow) hdg_ctx();
    if (!c) return fail(nullptr, HDG_E_ALLOC, "host allocation failed");
    c->physics = p->physics;
    c->precision = o->precision;
    c->nrhs = o->nrhs;
    c->k = kk;
    c->uniform = uniform;
    c->stab_scale = p->stab_scale;
    c->krylov_tol = o->krylov_tol > 0 ? o->krylov_tol : 1e-13;
    c->krylov_maxit = o->krylov_maxit > 0 ? o->krylov_maxit : 5000;
    c->refine_tol = o->refine_tol > 0 ? o->refine_tol : 1e-13;
    c->refine_maxit = o->refine_maxit > 0 ? o->refine_maxit : 10;
    c->refine_inner_tol = o->refine_inner_tol > 0 ? o->refine_inner_tol : 1e-6;
    c->cache_factors = o->cache_factors != 0;
    c->autotune = o->autotune != 0;
    if (o->autotune_table) c->tune_path = o->autotune_table;
    c->use_graph = o->use_graph != 0;
    c->graph_step = o->graph_step != 0;
    if ((o->dev_alloc == nullptr) != (o->dev_free == nullptr)) {
        g_init_err = "dev_alloc and dev_free: both or neither";
        delete c;
        return HDG_E_ARG;
    }
    c->dev_alloc = o->dev_alloc;
    c->dev_free = o->dev_free;
    c->alloc_user = o->alloc_user;
    if (o->precond != HDG_PC_JACOBI && o->precond != HDG_PC_SSOR) {
        g_init_err = "unknown precond";
        delete c;
        return HDG_E_ARG;
    }
    c->precond = o->precond;
    c->stream = (hipStream_t)stream;
    int st = build_mesh(c, m, p);
    if (st) {
        g_init_err = c->err;
        delete c;
        return st;
    }
    const int d = c->dim;
    if (!uniform) {
        if (c->physics != HDG_ACOUSTIC || d != 3) {
            g_init_err = "variable polynomial degree is built for 3D acoustics only";
            delete c;
            return HDG_E_UNSUPPORTED;
        }
        c->vardeg = true;
        c->degree.assign(m->degree, m->degree + m->n_elem);
        for (int64_t e = 0; e < c->n_elem; ++e) kk = std::max<int>(kk, c->degree[e]);
        c->k = kk;
    }
    c->fast_ac = c->physics == HDG_ACOUSTIC && !c->vardeg && c->nrhs == 1;
    c->m_local = (c->physics == HDG_ACOUSTIC) ? d + 1 : (c->physics == HDG_ELASTIC ? 9 : (c->physics == HDG_MAXWELL ? 6 : 7));
    c->m_trace = (c->physics == HDG_ACOUSTIC) ? 1 : (c->physics == HDG_ELASTIC ? 3 : 2);
    const int kface = c->vardeg ? var_face_degree() : kk;
    c->N = dim_p(kk, d);
    c->NF = dim_p(kface, d - 1);
    c->n_loc = c->m_local * c->N;
    c->bs = c->m_trace * c->NF;
    c->n_tr = (d + 1) * c->bs;
    c->n_local_dofs = c->n_elem * c->n_loc;
    c->n_trace_dofs = c->n_faces * c->bs;
    std::vector<int8_t> efnf, face_nf;
    std::vector<int32_t> cls[6];
    if (c->vardeg) {
        // face degree: the larger degree of the face's elements; compact local offsets
        std::vector<int> fk(c->n_faces, 0);
        for (int64_t F = 0; F < c->n_faces; ++F)
            for (int s2 = 0; s2 < 2; ++s2) {
                const int32_t e = c->face_elem[2 * F + s2];
                if (e >= 0) fk[F] = std::max<int>(fk[F], c->degree[e]);
            }
        face_nf.resize(c->n_faces);
        for (int64_t F = 0; F < c->n_faces; ++F) face_nf[F] = (int8_t)dim_p(fk[F], d - 1);
        efnf.resize(c->n_elem * (d + 1));
        for (int64_t i = 0; i < c->n_elem * (d + 1); ++i) efnf[i] = face_nf[c->elem_face[i]];
        c->loc_off_h.assign(c->n_elem + 1, 0);
        for (int64_t e = 0; e < c->n_elem; ++e) {
            c->loc_off_h[e + 1] = c->loc_off_h[e] + c->m_local * dim_p(c->degree[e], d);
            cls[c->degree[e]].push_back((int32_t)e);
        }
        c->n_local_dofs = c->loc_off_h[c->n_elem];
        for (int k = 1; k <= 5; ++k) c->cls_n[k] = (int64_t)cls[k].size();
    }
    c->K_sign = (c->physics == HDG_ACOUSTIC) ? -1.0 : 1.0;
    // densely factored (Schur) block: acoustic p, elastic v, maxwell E
    c->Ns = (c->physics == HDG_ACOUSTIC) ? c->N : (c->physics == HDG_MAXWELL_GLM ? 4 * c->N : 3 * c->N);
    c->s_row0 = (c->physics == HDG_ACOUSTIC) ? d * c->N : (c->physics == HDG_ELASTIC ? 6 * c->N : 3 * c->N);
    if (!supported(c)) {
        std::ostringstream os;
        os << "configuration not built: physics " << c->physics << ", k " << kk << ", nrhs " << c->nrhs;
        g_init_err = os.str();
        delete c;
        return HDG_E_UNSUPPORTED;
    }
    if (c->graph_step && c->precision != HDG_FP64) {
        g_init_err = "graph_step: FP64 only (the refinement of the mixed precisions decides on the host)";
        delete c;
        return HDG_E_UNSUPPORTED;
    }
    // reference tables
    build_ref_tables(d, kk, c->ref);
    build_face_tables(d, kk, kface, c->reff);

    int s = 0;
#define TRY(x)                       \
    do {                             \
        if ((s = (x)) != HDG_OK) {   \
            g_init_err = c->err;     \
            hdg_destroy(c);          \
            return s;                \
        }                            \
    } while (0)
    TRY(upload(c, &c->d_geom, c->geom));
    TRY(upload(c, &c->d_eface, c->elem_face));
    TRY(upload(c, &c->d_eperm, c->elem_perm));
    TRY(upload(c, &c->d_face_elem, c->face_elem));
    TRY(upload(c, &c->d_face_lf, c->face_lf));
    TRY(upload(c, &c->d_face_bnd, c->face_bnd));
    if (c->precond == HDG_PC_SSOR) {
        // greedy colouring of the faces in face order: faces that share an element (a nonzero
        // off-diagonal block of K) get different colours, so the faces of one colour are
        // independent in a Gauss-Seidel sweep
        const int nv = c->dim + 1;
        std::vector<int8_t> color(c->n_faces, -1);
        int nc = 0;
        for (int64_t F = 0; F < c->n_faces; ++F) {
            unsigned used = 0;
            for (int s2 = 0; s2 < 2; ++s2) {
                const int32_t e = c->face_elem[2 * F + s2];
                if (e < 0) continue;
                for (int q = 0; q < nv; ++q) {
                    const int32_t G = c->elem_face[(int64_t)e * nv + q];
                    if (G != F && color[G] >= 0) used |= 1u << color[G];
                }
            }
            int col = 0;
            while (used & (1u << col)) ++col;
            color[F] = (int8_t)col;
            nc = std::max(nc, col + 1);
        }
        // the colouring is a proper edge colouring of the element graph (elements joined by their
        // faces); greedy leaves a few faces in colour nv (one above the element degree).  Each
        // such face F between elements u and v misses one colour al at u and one colour be at v;
        // swapping al and be along the chain of faces coloured al, be that starts at v frees al at
        // v unless the chain ends at u (Kempe's interchange).  When every face leaves colour nv,
        // one sweep launch per direction goes.
        if (nc == nv + 1) {
            auto other = [&](int32_t G, int32_t e) {
                const int32_t e0 = c->face_elem[2 * G], e1 = c->face_elem[2 * G + 1];
                return e0 == e ? e1 : e0;
            };
            auto face_of = [&](int32_t e, int col) -> int32_t {
                for (int q = 0; q < nv; ++q) {
                    const int32_t G = c->elem_face[(int64_t)e * nv + q];
                    if (color[G] == col) return G;
                }
                return -1;
            };
            auto missing = [&](int32_t e, int32_t F) {
                unsigned used = 0;
                for (int q = 0; q < nv; ++q) {
                    const int32_t G = c->elem_face[(int64_t)e * nv + q];
                    if (G != F) used |= 1u << color[G];
                }
                int col = 0;
                while (used & (1u << col)) ++col;
                return col;
            };
            bool left = false;
            std::vector<int32_t> chain;
            for (int64_t F = 0; F < c->n_faces; ++F) {
                if (color[F] != nv) continue;
                const int32_t u = c->face_elem[2 * F], v = c->face_elem[2 * F + 1];
                if (u < 0 || v < 0) {
                    left = true;
                    continue;
                }
                const int al = missing(u, (int32_t)F), be = missing(v, (int32_t)F);
                if (al >= nv || be >= nv) {   // cannot happen for interior faces of simplices
                    left = true;
                    continue;
                }
                if (al == be) {
                    color[F] = (int8_t)al;
                    continue;
                }
                // chain from v: its al-face, then the be-face of the next element, ...
                chain.clear();
                int32_t e = v;
                int col = al;
                bool hits_u = false;
                for (int64_t len = 0; len < c->n_faces; ++len) {   // a path: it ends
                    const int32_t G = face_of(e, col);
                    if (G < 0) break;
                    chain.push_back(G);
                    e = other(G, e);
                    if (e < 0) break;
                    if (e == u) {
                        hits_u = true;
                        break;
                    }
                    col = col == al ? be : al;
                }
                if (hits_u) {
                    left = true;
                    continue;
                }
                for (int32_t G : chain) color[G] = (int8_t)(color[G] == al ? be : al);
                color[F] = (int8_t)al;
            }
            if (!left) nc = nv;
        }
        c->ncolors = nc;
        c->color_off.assign(nc + 1, 0);
        for (int64_t F = 0; F < c->n_faces; ++F) ++c->color_off[color[F] + 1];
        for (int k2 = 0; k2 < nc; ++k2) c->color_off[k2 + 1] += c->color_off[k2];
        std::vector<int32_t> cf(c->n_faces);
        std::vector<int64_t> pos(c->color_off.begin(), c->color_off.end() - 1);
        for (int64_t F = 0; F < c->n_faces; ++F) cf[pos[color[F]]++] = (int32_t)F;
        // the off-diagonal blocks in sweep order: for every position of the colour order the
        // blocks of its lower-colour neighbours (the forward sweep's), then, after all of those,
        // the blocks of the higher-colour neighbours (the backward sweep's).  A sweep launch over
        // the faces of one colour then streams one contiguous range of blocks.
        const int ns1 = c->nslot - 1;
        std::vector<int32_t> off(2 * (c->n_faces + 1)), nb, dst(c->n_faces * ns1, -1);
        nb.reserve(c->n_faces * ns1);
        for (int dir = 0; dir < 2; ++dir) {
            int32_t* o = off.data() + dir * (c->n_faces + 1);
            for (int64_t p = 0; p < c->n_faces; ++p) {
                const int32_t F = cf[p];
                o[p] = (int32_t)nb.size();
                for (int sl = 1; sl < c->nslot; ++sl) {
                    const int32_t G = c->bsr_cols_h[F * c->nslot + sl];
                    if (G < 0 || (color[G] < color[F]) != (dir == 0)) continue;
                    dst[F * ns1 + sl - 1] = (int32_t)nb.size();
                    nb.push_back(G);
                }
            }
            o[c->n_faces] = (int32_t)nb.size();
        }
        c->ss_nblk = (int64_t)nb.size();
        TRY(upload(c, &c->d_cfaces, cf));
        TRY(upload(c, &c->d_ssoff, off));
        TRY(upload(c, &c->d_ssdst, dst));
        if (!nb.empty()) TRY(upload(c, &c->d_ssnb, nb));
    }
    TRY(upload(c, &c->d_bsr_cols, c->bsr_cols_h));
    TRY(upload(c, &c->tab.Sr, c->ref.Sr));
    TRY(upload(c, &c->tab.Mf, c->ref.Mf));
    TRY(upload(c, &c->tab.Tsym, c->ref.Tsym));
    TRY(upload(c, &c->tab.Ef, c->reff.E));
    TRY(upload_f32(c, &c->tab.Sr32, c->ref.Sr));
    TRY(upload_f32(c, &c->tab.Mf32, c->ref.Mf));
    TRY(upload_f32(c, &c->tab.Tsym32, c->ref.Tsym));
    TRY(upload_f32(c, &c->tab.Ef32, c->reff.E));
    TRY(upload(c, &c->tab.Tfull, c->ref.Tfull));
    TRY(upload_f32(c, &c->tab.Tfull32, c->ref.Tfull));
    TRY(upload_transposed(c, c->tab, c->ref, c->reff));
    if (c->vardeg) {
        std::vector<int8_t> edeg(c->degree.begin(), c->degree.end());
        TRY(upload(c, &c->d_loc_off, c->loc_off_h));
        TRY(upload(c, &c->d_efnf, efnf));
        TRY(upload(c, &c->d_face_nf, face_nf));
        TRY(upload(c, &c->d_edeg, edeg));
        for (int k = 1; k <= 5; ++k) {
            if (!c->cls_n[k]) continue;
            TRY(upload(c, &c->d_cls[k], cls[k]));
            RefTables rk;
            RefFaceTables ek;
            build_ref_tables(d, k, rk);
            build_face_tables(d, k, kface, ek);
            TRY(upload_tables(c, c->tabk[k], rk, ek));
        }
    }
    if (c->physics == HDG_MAXWELL || c->physics == HDG_MAXWELL_GLM) {
        std::vector<double> ef(c->n_elem * (d + 1) * 6);
        for (int64_t e = 0; e < c->n_elem; ++e)
            for (int f = 0; f <= d; ++f)
                for (int q = 0; q < 6; ++q)
                    ef[(e * (d + 1) + f) * 6 + q] = c->frame[(int64_t)c->elem_face[e * (d + 1) + f] * 6 + q];
        TRY(upload(c, &c->d_eframe, ef));
    }


    const size_t tsz = (c->precision == HDG_FP64) ? sizeof(double) : sizeof(float);
    const int64_t ne = c->n_elem, R = c->nrhs;
    TRY(dalloc(c, (char**)&c->d_Ke, ne * c->n_tr * c->n_tr * tsz));
    TRY(dalloc(c, (char**)&c->d_re, ne * c->n_tr * R * tsz));
    TRY(dalloc(c, (char**)&c->d_Zt, ne * c->n_tr * c->Ns * tsz));
    TRY(dalloc(c, (char**)&c->d_z, ne * c->n_loc * R * tsz));
    if (c->precision != HDG_FP64 || c->cache_factors)
        TRY(dalloc(c, (char**)&c->d_LU, ne * c->Ns * c->Ns * tsz));
    TRY(dalloc(c, &c->d_status, 1));
    const int64_t ntr = c->n_trace_dofs;
    TRY(dalloc(c, &c->d_bsr, c->n_faces * c->nslot * c->bs * c->bs));
    if (c->precision != HDG_FP64 && (R == 1 || R == 32) && c->nslot == 7)
        TRY(dalloc(c, &c->d_bsr32, c->n_faces * c->nslot * c->bs * c->bs));
    TRY(dalloc(c, &c->d_rhs, ntr * R));
    TRY(dalloc(c, &c->d_pinv, c->n_faces * c->bs * c->bs));
    TRY(dalloc(c, &c->d_cg_r, ntr * R));
    TRY(dalloc(c, &c->d_cg_z, ntr * R));
    TRY(dalloc(c, &c->d_cg_p, ntr * R));
    TRY(dalloc(c, &c->d_cg_q, std::max<int64_t>(ntr * R, c->n_faces * c->bs * c->bs)));
    c->red_blocks = 1024;
    TRY(dalloc(c, &c->d_red, (int64_t)RED_MAX * 32));
    TRY(dalloc(c, &c->d_scal, 8 * 32));
    TRY(dalloc(c, &c->d_cgflags, 8));
    const int64_t nl = c->n_local_dofs * R;
    if (c->precision != HDG_FP64) {
        TRY(dalloc(c, &c->d_f_saved, nl));
        TRY(dalloc(c, &c->d_lbnd_saved, ntr * R));
        TRY(dalloc(c, &c->d_du, nl));
        TRY(dalloc(c, &c->d_dlam, ntr * R));
        TRY(dalloc(c, &c->d_re64, ne * c->n_tr * R));
        TRY(dalloc(c, &c->d_sq, std::max<int64_t>(3 * ne, ne * R)));
    }
    if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_rr, hipEventDisableTiming) != hipSuccess) {
        g_init_err = "hipEventCreate failed";
        hdg_destroy(c);
        return HDG_E_HIP;
    }
    if (hipHostMalloc((void**)&c->h_rr, 32 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        c->h_rr = nullptr;
        g_init_err = "hipHostMalloc failed";
        hdg_destroy(c);
        return HDG_E_HIP;
    }
    if (c->graph_step &&
        hipStreamCreateWithFlags(&c->sg_stream, hipStreamNonBlocking) != hipSuccess) {
        c->sg_stream = nullptr;
        g_init_err = "stream creation for the step graph failed";
        hdg_destroy(c);
        return HDG_E_HIP;
    }
    if (c->use_graph && c->vardeg) {
        bool ok = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) == hipSuccess &&
                  hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) == hipSuccess &&
                  hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming) == hipSuccess;
        for (int i = 0; i < 6 && ok; ++i)
            ok = hipStreamCreateWithFlags(&c->side[i], hipStreamNonBlocking) == hipSuccess &&
                 hipEventCreateWithFlags(&c->ev_join[i], hipEventDisableTiming) == hipSuccess;
        if (!ok) {
            g_init_err = "stream or event creation for the condensation graph failed";
            hdg_destroy(c);
            return HDG_E_HIP;
        }
    }
    {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
            c->device_name = prop.gcnArchName;
            const size_t colon = c->device_name.find(':');
            if (colon != std::string::npos) c->device_name.resize(colon);
        }
        if (c->device_name.empty()) c->device_name = "unknown";
    }
    if (!c->tune_path.empty()) read_tune_table(c);
    if (static_scratch_setup() != HDG_OK) {   // address of the no-allocation solve's scratch
        g_init_err = "hipGetSymbolAddress of the static trace-solve scratch failed";
        hdg_destroy(c);
        return HDG_E_HIP;
    }
#undef TRY
    *out = c;
    return HDG_OK;
}

hdg_status hdg_query(const hdg_ctx* c, int key, int64_t* v) {
    if (!c || !v) return HDG_E_ARG;
    switch (key) {
        case HDG_Q_N_ELEM: *v = c->n_elem; break;
        case HDG_Q_N_FACES: *v = c->n_faces; break;
        case HDG_Q_N_BFACES: *v = c->n_bfaces; break;
        case HDG_Q_N_LOCAL_DOFS: *v = c->n_local_dofs; break;
        case HDG_Q_N_TRACE_DOFS: *v = c->n_trace_dofs; break;
        case HDG_Q_N_VOL_POINTS: {
            std::vector<double> p, w;
            simplex_quadrature(c->dim, c->k + 2, p, w);
            *v = c->n_elem * (int64_t)w.size();
            break;
        }
        case HDG_Q_N_BND_POINTS: {
            std::vector<double> p, w;
            simplex_quadrature(c->dim - 1, c->k + 3, p, w);
            *v = c->n_bfaces * (int64_t)w.size();
            break;
        }
        case HDG_Q_LAST_ITERS: *v = c->last_iters; break;
        case HDG_Q_LAST_REFINE: *v = c->last_refine; break;
        case HDG_Q_M_LOCAL: *v = c->m_local; break;
        case HDG_Q_M_TRACE: *v = c->m_trace; break;
        case HDG_Q_STEP_GRAPH: *v = c->sg_replayed ? 1 : 0; break;
        case HDG_Q_STEP_GRAPH_ITERS: *v = c->sgexec ? c->sg_nit : 0; break;
        case HDG_Q_N_COLORS: *v = c->ncolors; break;
        case HDG_Q_SCHEDULE: {
            const int pi = c->precision == HDG_FP64 ? 1 : 0;
            int64_t x = 0;
            for (int k = 1; k <= 5; ++k)
                if (c->sched[pi][k] >= 0 && (c->vardeg ? c->cls_n[k] > 0 : k == c->k))
                    x |= (int64_t)(c->sched[pi][k] + 1) << (4 * (k - 1));
            *v = x;
            break;
        }
        default: return HDG_E_ARG;
    }
    return HDG_OK;
}

hdg_status hdg_condense(hdg_ctx* c, double a, const double* f_loc, const double* lam_bnd) {
    if (!c) return HDG_E_ARG;
    if (!f_loc || !lam_bnd) return fail(c, HDG_E_ARG, "null f_loc or lam_bnd");
    if (!(a > 0) || !std::isfinite(a)) return fail(c, HDG_E_ARG, "stage coefficient must be positive");
    HIPCHK(hipMemsetAsync(c->d_status, 0, sizeof(int), c->stream));
    const int64_t R = c->nrhs;
    if (c->precision != HDG_FP64) {   // kept for the FP64 refinement residuals
        HIPCHK(hipMemcpyAsync(c->d_f_saved, f_loc, c->n_local_dofs * R * sizeof(double),
                              hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(c->d_lbnd_saved, lam_bnd, c->n_trace_dofs * R * sizeof(double),
                              hipMemcpyDeviceToDevice, c->stream));
    }
    int e;
    {
        EventTimer t(c, &c->tim.condense);
        e = c->fast_ac ? launch_condense_acoustic(c, a, f_loc) : launch_condense_general(c, a, f_loc);
    }
    if (e) return fail(c, HDG_E_HIP, "condensation kernel launch failed");
    {
        EventTimer t(c, &c->tim.assemble);
        e = launch_assemble(c, lam_bnd);
        // block SSOR (the trace solve and the refinement's correction solves) uses neither the
        // block-Jacobi inverses nor the FP32 copy of K; a later Jacobi solve forms them itself
        if (!(c->precond == HDG_PC_SSOR && ssor_supported(c))) {
            if (!e) e = launch_block_inverse(c);
            if (!e) e = launch_bsr_f32(c);
        }
    }
    if (e) return fail(c, HDG_E_HIP, "assembly kernel launch failed");
    c->last_a = a;
    c->condensed = true;
    c->z_consumed = false;
    c->factors_cached = c->d_LU != nullptr && c->nrhs == 1;
    return HDG_OK;
}

hdg_status hdg_condense_rhs(hdg_ctx* c, double a, const double* f_loc, const double* lam_bnd) {
    if (!c) return HDG_E_ARG;
    if (!f_loc || !lam_bnd) return fail(c, HDG_E_ARG, "null f_loc or lam_bnd");
    if (c->nrhs != 1) return fail(c, HDG_E_UNSUPPORTED, "right-hand-side condensation: one right-hand side");
    if (!c->condensed || !c->factors_cached)
        return fail(c, HDG_E_STATE, "hdg_condense_rhs needs the factors of an earlier hdg_condense (FP64: cache_factors)");
    if (a != c->last_a) return fail(c, HDG_E_STATE, "hdg_condense_rhs: stage coefficient differs from the factored one");
    const int64_t R = c->nrhs;
    if (c->precision != HDG_FP64) {   // kept for the FP64 refinement residuals
        HIPCHK(hipMemcpyAsync(c->d_f_saved, f_loc, c->n_local_dofs * R * sizeof(double),
                              hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(c->d_lbnd_saved, lam_bnd, c->n_trace_dofs * R * sizeof(double),
                              hipMemcpyDeviceToDevice, c->stream));
    }
    int e;
    {
        EventTimer t(c, &c->tim.condense);
        e = c->fast_ac ? launch_condense_rhs_acoustic(c, a, f_loc) : launch_condense_rhs_general(c, f_loc);
    }
    if (e) return fail(c, HDG_E_HIP, "right-hand-side condensation launch failed");
    {
        EventTimer t(c, &c->tim.assemble);
        e = launch_assemble_rhs(c, lam_bnd);
    }
    if (e) return fail(c, HDG_E_HIP, "right-hand-side assembly launch failed");
    c->z_consumed = false;
    return HDG_OK;
}

hdg_status hdg_trace_solve(hdg_ctx* c, double* lambda, int* iters, double* relres) {
    if (!c) return HDG_E_ARG;
    if (!lambda) return fail(c, HDG_E_ARG, "null lambda");
    if (!c->condensed) return fail(c, HDG_E_STATE, "hdg_trace_solve before hdg_condense");
    int s = check_status(c);
    if (s) return s;
    int r;
    {
        EventTimer t(c, &c->tim.solve);
        // mixed precision: K already carries the FP32 factors' error and the refinement's FP64
        // residual removes it, so the products may read the FP32 copy as well
        r = (c->precond == HDG_PC_SSOR && ssor_supported(c))
                ? trace_cg_ssor(c, lambda, c->krylov_tol, iters, relres)
                : trace_cg(c, lambda, c->krylov_tol, iters, relres, c->d_bsr32 != nullptr);
    }
    if (r == HDG_E_NOCONV) return fail(c, r, "trace solve did not reach krylov_tol");
    if (r) return fail(c, r, "trace solve failed");
    return HDG_OK;
}

hdg_status hdg_trace_solve_static(hdg_ctx* c, double* lambda, int* iters, double* relres) {
    if (!c) return HDG_E_ARG;
    if (!lambda) return fail(c, HDG_E_ARG, "null lambda");
    const int64_t need = trace_static_need(c);
    if (need > TRACE_STATIC_DOUBLES) {
        std::ostringstream os;
        os << "hdg_trace_solve_static: this system needs " << need * 8 << " bytes of scratch, the static "
           << "scratch holds " << TRACE_STATIC_DOUBLES * 8 << " bytes (use hdg_trace_solve)";
        return fail(c, HDG_E_ARG, os.str());
    }
    if (!c->condensed) return fail(c, HDG_E_STATE, "hdg_trace_solve_static before hdg_condense");
    int s = check_status(c);
    if (s) return s;
    int r;
    {
        EventTimer t(c, &c->tim.solve);
        r = trace_cg_static(c, lambda, iters, relres);
    }
    if (r == HDG_E_NOCONV) return fail(c, r, "trace solve did not reach krylov_tol");
    if (r) return fail(c, r, "trace solve failed");
    return HDG_OK;
}

// Mixed-precision refinement (iterative refinement of the full stage system): the residual of
// the full uncondensed system [A B; C D] (u, lam) = (f, g) is evaluated in FP64 from the element
// operators, corrected through the FP32 factors and an FP64 trace solve, until the measured FP64
// residual of every right-hand-side column satisfies
//     |s| <= refine_tol |(f, lam_D)|,
// s = (f - A u - B lam, -(C u + D lam)) over the local rows and the trace rows of the
// non-Dirichlet faces (the Dirichlet rows lam = lam_D hold exactly), (f, lam_D) the right-hand
// side of the full system.  Each correction is followed by a check pass that forms this residual
// at the corrected iterate; a full residual pass (which also forms the next correction's
// right-hand side) runs only when the check fails.  The inner trace solves run to
// refine_inner_tol; an inner solve that stops short of it still yields a correction, whose effect
// the next check measures, so it is not an error by itself; a residual that does not halve from
// one correction to the next is (HDG_E_NOCONV), as is refine_maxit corrections without meeting
// the test.

// |(f, lam_D)| per column, the scale of the relative residual
static int refine_scale(hdg_ctx* c, std::vector<double>& scale) {
    const int R = c->nrhs;
    std::vector<double> fs(R), bs(R);
    if (launch_col_sq(c, c->n_local_dofs, R, c->d_f_saved, fs.data()) ||
        launch_col_sq(c, c->n_faces * c->bs, R, c->d_lbnd_saved, bs.data(), true))
        return fail(c, HDG_E_HIP, "refinement norm reduction failed");
    scale.assign(R, 1.0);
    for (int r = 0; r < R; ++r) {
        const double v = std::sqrt(fs[r] + bs[r]);
        scale[r] = v > 0.0 ? v : 1.0;
    }
    return HDG_OK;
}

// Relative residual per column after a check pass: elem_nrm holds |s| of the local rows per
// element (and column), re64 the element parts -t_e of the trace rows.  Returns the largest.
static int refine_residual(hdg_ctx* c, const double* elem_nrm, const std::vector<double>& scale, double* worst) {
    const int R = c->nrhs;
    std::vector<double> lo(R), tr(R);
    if (launch_assemble_rhs64(c, c->d_re64, c->d_lbnd_saved) ||
        launch_col_sq(c, c->n_elem, R, elem_nrm, lo.data()) ||
        launch_col_sq(c, c->n_faces * c->bs, R, c->d_rhs, tr.data()))
        return fail(c, HDG_E_HIP, "refinement residual reduction failed");
    double w = 0.0;
    bool finite = true;
    for (int r = 0; r < R; ++r) {
        const double v = std::sqrt(lo[r] + tr[r]) / scale[r];
        c->last_resid[r] = v;
        if (!(v - v == 0.0)) finite = false;
        else w = std::max(w, v);
    }
    c->has_resid = true;
    *worst = finite ? w : std::numeric_limits<double>::quiet_NaN();
    return HDG_OK;
}

// Verdict after the check of correction `it` (residual res, previous res prev): HDG_OK when
// converged, -1 to continue, or an error.
static int refine_verdict(hdg_ctx* c, int it, double res, double prev) {
    c->last_refine = it;
    if (!(res == res)) return fail(c, HDG_E_NOCONV, "refinement produced a non-finite residual");
    if (res <= c->refine_tol) return HDG_OK;
    if (it > 1 && res > 0.5 * prev) return fail(c, HDG_E_NOCONV, "refinement stagnated");
    if (it == c->refine_maxit) return fail(c, HDG_E_NOCONV, "refinement did not reach refine_tol within refine_maxit");
    return -1;
}

// correction trace solve: lam += dlam with K dlam = (assembled re64)
static int refine_trace_step(hdg_ctx* c, double* lambda, float* t_sol) {
    const int64_t nt = c->n_trace_dofs * c->nrhs;
    int r;
    {
        EventTimer t(c, t_sol);
        if (launch_assemble_rhs64(c, c->d_re64, c->d_lbnd_saved)) return fail(c, HDG_E_HIP, "refinement assembly launch failed");
        HIPCHK(hipMemsetAsync(c->d_dlam, 0, nt * sizeof(double), c->stream));
        int its;
        double rr;
        // block SSOR when configured (the FP64 scaled matrix of the first solve), else block
        // Jacobi with the products on the FP32 copy of K
        r = (c->precond == HDG_PC_SSOR && ssor_supported(c))
                ? trace_cg_ssor(c, c->d_dlam, c->refine_inner_tol, &its, &rr)
                : trace_cg(c, c->d_dlam, c->refine_inner_tol, &its, &rr, true);
    }
    if (r && r != HDG_E_NOCONV) return fail(c, r, "refinement trace solve failed");
    if (launch_axpy(c, nt, 1.0, c->d_dlam, lambda)) return fail(c, HDG_E_HIP, "refinement update launch failed");
    return HDG_OK;
}

// Acoustic mixed precision: recovery and refinement fused per element (the velocity is
// recovered in closed form in FP64, so the velocity rows of the residual vanish and the
// iteration runs on (p, lam)).  First pass: recovery from the FP32 factors, FP64 residual and
// the first correction's right-hand side.  Each correction pass applies the correction and
// checks the residual of the corrected iterate.
static hdg_status recover_refine_acoustic(hdg_ctx* c, double* lambda, double* u) {
    const int64_t ne = c->n_elem;
    int e;
    {
        EventTimer t(c, &c->tim.recover);
        e = launch_refine_acoustic(c, lambda, lambda, 1, 1, u, c->d_sq);
    }
    if (e) return fail(c, HDG_E_HIP, "recovery kernel launch failed");
    c->z_consumed = true;
    std::vector<double> scale;
    int s = refine_scale(c, scale);
    if (s) return s;
    double prev = 0.0;
    for (int it = 1; it <= c->refine_maxit; ++it) {
        float t_sol = 0.f, t_el = 0.f, t_res = 0.f;
        if ((s = refine_trace_step(c, lambda, &t_sol))) return s;
        {
            EventTimer t(c, &t_el);
            e = launch_refine_acoustic(c, lambda, c->d_dlam, 0, 2, u, c->d_sq);
        }
        if (e) return fail(c, HDG_E_HIP, "refinement kernel launch failed");
        double res;
        {
            EventTimer t(c, &t_res);
            if ((s = refine_residual(c, c->d_sq + 2 * ne, scale, &res))) return s;
        }
        c->tim.refine_elem += t_el;
        c->tim.refine_solve += t_sol + t_res;
        const int v = refine_verdict(c, it, res, prev);
        if (v >= 0) return v;
        prev = res;
        {   // full residual of the current iterate (no correction): next right-hand side
            EventTimer t(c, &t_el);
            e = launch_refine_acoustic(c, lambda, c->d_dlam, 2, 1, u, c->d_sq);
        }
        if (e) return fail(c, HDG_E_HIP, "refinement kernel launch failed");
        c->tim.refine_elem += t_el;
    }
    return fail(c, HDG_E_NOCONV, "refinement did not reach refine_tol within refine_maxit");
}

hdg_status hdg_recover(hdg_ctx* c, double* lambda, double* u) {
    if (!c) return HDG_E_ARG;
    if (!lambda || !u) return fail(c, HDG_E_ARG, "null lambda or u");
    if (!c->condensed) return fail(c, HDG_E_STATE, "hdg_recover before hdg_condense");
    if (c->z_consumed)
        return fail(c, HDG_E_STATE, "mixed precision: the refinement of the previous hdg_recover used the "
                                    "condensation buffers; call hdg_condense again");
    int s = check_status(c);
    if (s) return s;
    c->last_refine = 0;
    c->has_resid = false;
    c->tim.refine_elem = 0.f;
    c->tim.refine_solve = 0.f;
    if (c->precision != HDG_FP64 && c->fast_ac) return recover_refine_acoustic(c, lambda, u);
    int e;
    {
        EventTimer t(c, &c->tim.recover);
        e = c->fast_ac ? launch_refine_acoustic(c, lambda, lambda, 1, 0, u, nullptr)
                       : launch_recover_any(c, lambda, u);
    }
    if (e) return fail(c, HDG_E_HIP, "recovery kernel launch failed");
    if (c->precision == HDG_FP64) return HDG_OK;

    // Iterative refinement of the full stage system (see above), element work in separate passes:
    // residual (and correction right-hand side), trace solve, recovery of the correction.
    c->z_consumed = true;
    const int64_t nl = c->n_local_dofs * c->nrhs;
    std::vector<double> scale;
    if ((s = refine_scale(c, scale))) return s;
    {
        float t_res = 0.f;
        {
            EventTimer t(c, &t_res);
            e = launch_refine_general(c, u, lambda, false, nullptr);
        }
        if (e) return fail(c, HDG_E_HIP, "refinement kernel launch failed");
        c->tim.refine_elem += t_res;
    }
    double prev = 0.0;
    for (int it = 1; it <= c->refine_maxit; ++it) {
        float t_sol = 0.f, t_rec = 0.f, t_chk = 0.f, t_res = 0.f;
        if ((s = refine_trace_step(c, lambda, &t_sol))) return s;
        {
            EventTimer t(c, &t_rec);
            e = launch_recover_any(c, c->d_dlam, c->d_du);
            if (!e) e = launch_axpy(c, nl, 1.0, c->d_du, u);
        }
        if (e) return fail(c, HDG_E_HIP, "refinement recovery launch failed");
        {
            EventTimer t(c, &t_chk);
            e = launch_refine_general(c, u, lambda, true, c->d_sq);
        }
        if (e) return fail(c, HDG_E_HIP, "refinement check launch failed");
        double res;
        {
            EventTimer t(c, &t_res);
            if ((s = refine_residual(c, c->d_sq, scale, &res))) return s;
        }
        c->tim.refine_elem += t_rec + t_chk;
        c->tim.refine_solve += t_sol + t_res;
        const int v = refine_verdict(c, it, res, prev);
        if (v >= 0) return v;
        prev = res;
        {
            float t_full = 0.f;
            {
                EventTimer t(c, &t_full);
                e = launch_refine_general(c, u, lambda, false, nullptr);
            }
            if (e) return fail(c, HDG_E_HIP, "refinement kernel launch failed");
            c->tim.refine_elem += t_full;
        }
    }
    return fail(c, HDG_E_NOCONV, "refinement did not reach refine_tol within refine_maxit");
}

hdg_status hdg_last_residual(const hdg_ctx* c, double* rel) {
    if (!c || !rel) return HDG_E_ARG;
    if (!c->has_resid) return HDG_E_STATE;
    for (int r = 0; r < c->nrhs; ++r) rel[r] = c->last_resid[r];
    return HDG_OK;
}

hdg_status hdg_apply_mass(hdg_ctx* c, double a, const double* u, double* f) {
    if (!c) return HDG_E_ARG;
    if (!u || !f) return fail(c, HDG_E_ARG, "null pointer");
    if (launch_apply_mass(c, a, u, f)) return fail(c, HDG_E_HIP, "mass kernel launch failed");
    return HDG_OK;
}

}  // extern "C"

namespace {
// Butcher tableau of the scheme and the inverse d = A^{-1} of its (lower-triangular) matrix
int step_tableau(int scheme, double Dm[3][3]) {
    double A[3][3] = {};
    int ns = 1;
    if (scheme == HDG_BACKWARD_EULER) {
        A[0][0] = 1.0;
    } else {
        ns = 3;
        // gamma: root in (1/6, 1/2) of x^3 - 3x^2 + 3x/2 - 1/6 (Newton from 0.4)
        double g = 0.4;
        for (int it = 0; it < 60; ++it) {
            double fx = ((g - 3.0) * g + 1.5) * g - 1.0 / 6.0;
            double dfx = (3.0 * g - 6.0) * g + 1.5;
            g -= fx / dfx;
        }
        double b1 = -1.5 * g * g + 4.0 * g - 0.25, b2 = 1.5 * g * g - 5.0 * g + 1.25;
        A[0][0] = g;
        A[1][0] = 0.5 * (1.0 - g);
        A[1][1] = g;
        A[2][0] = b1;
        A[2][1] = b2;
        A[2][2] = g;
    }
    for (int i = 0; i < ns; ++i) {   // forward substitution for the lower-triangular inverse
        for (int j = 0; j < 3; ++j) Dm[i][j] = 0.0;
        Dm[i][i] = 1.0 / A[i][i];
        for (int j = 0; j < i; ++j) {
            double acc = 0.0;
            for (int m = j; m < i; ++m) acc += A[i][m] * Dm[m][j];
            Dm[i][j] = -acc / A[i][i];
        }
    }
    return ns;
}

// stage glue of stage i: d_fstage = a Mw u*_i (+ src), u*_i = u^n - (1/d_ii) sum_{j<i} d_ij (U_j - u^n)
int stage_rhs(hdg_ctx* c, int i, const double Dm[3][3], double dt, const double* u, const double* src) {
    const int64_t nl = c->n_local_dofs * c->nrhs;
    const double a = Dm[i][i] / dt;
    int e = launch_lincomb(c, nl, 1.0, u, 0.0, nullptr, c->d_ustar);
    double wsum = 0.0;
    for (int j = 0; j < i && !e; ++j) {
        const double w = -Dm[i][j] / Dm[i][i];
        wsum += w;
        e = launch_axpy(c, nl, w, c->d_stage + j * nl, c->d_ustar);
    }
    if (!e && wsum != 0.0) e = launch_axpy(c, nl, -wsum, u, c->d_ustar);
    if (!e) e = launch_apply_mass(c, a, c->d_ustar, c->d_fstage);
    if (!e && src) e = launch_axpy(c, nl, 1.0, src, c->d_fstage);
    return e;
}

// The launches of one whole step with no host synchronisation, for capture: stage glue,
// condensation (of the right-hand side only when `reuse`), the device-side CG with `nit`
// iterations, recovery into the stage buffer.  FP64 only.
int step_launches(hdg_ctx* c, int ns, const double Dm[3][3], double dt, const double* u, double* lambda,
                  const double* lam_bnd, const double* src, bool reuse, int nit) {
    const int64_t nl = c->n_local_dofs * c->nrhs;
    const int64_t nt = c->n_trace_dofs * c->nrhs;
    int e = launch_zero_ints(c, c->d_status, 1);
    for (int i = 0; i < ns && !e; ++i) {
        const double a = Dm[i][i] / dt;
        const double* lb = lam_bnd + i * nt;
        e = stage_rhs(c, i, Dm, dt, u, src);
        if (e) break;
        if (reuse) {
            e = c->fast_ac ? launch_condense_rhs_acoustic(c, a, c->d_fstage)
                           : launch_condense_rhs_general(c, c->d_fstage);
            if (!e) e = launch_assemble_rhs(c, lb);
        } else {
            e = c->fast_ac ? launch_condense_acoustic(c, a, c->d_fstage) : launch_condense_general(c, a, c->d_fstage);
            if (!e) e = launch_assemble(c, lb);
        }
        // the preconditioner's data (block-Jacobi inverses, or the scaled SSOR matrix) are formed
        // by the solve after each assembly
        if (!e)
            e = (c->precond == HDG_PC_SSOR && ssor_supported(c) && c->nrhs == 1)
                    ? trace_cg_ssor_device(c, lambda, c->krylov_tol, nit, c->d_cgflags + 2 * i, c->d_scal + 160 + i)
                    : trace_cg_device(c, lambda, c->krylov_tol, nit, c->d_cgflags + 2 * i, c->d_scal + 160 + i);
        if (!e) e = launch_recover_any(c, lambda, c->d_stage + i * nl);
    }
    return e;
}

// capture the step into c->sgexec (nothing runs); the vardeg condensation graph is not nested
int capture_step(hdg_ctx* c, int ns, const double Dm[3][3], double dt, const double* u, double* lambda,
                 const double* lam_bnd, const double* src, bool reuse, int nit) {
    if (c->sgexec) {
        (void)hipGraphExecDestroy(c->sgexec);
        c->sgexec = nullptr;
    }
    if (hipStreamBeginCapture(c->sg_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return -1;
    hipStream_t user = c->stream;
    const bool ug = c->use_graph;
    c->stream = c->sg_stream;
    c->use_graph = false;
    const int e = step_launches(c, ns, Dm, dt, u, lambda, lam_bnd, src, reuse, nit);
    c->stream = user;
    c->use_graph = ug;
    hipGraph_t graph = nullptr;
    const hipError_t ee = hipStreamEndCapture(c->sg_stream, &graph);
    if (e || ee != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        return e ? e : (int)ee;
    }
    const hipError_t ie = hipGraphInstantiate(&c->sgexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) {
        c->sgexec = nullptr;
        return (int)ie;
    }
    c->sg_reuse = reuse;
    c->sg_nit = nit;
    return 0;
}
}  // namespace

extern "C" {
hdg_status hdg_step(hdg_ctx* c, double t, double dt, int scheme, double* u, double* lambda,
                    const double* lam_bnd, const double* src) {
    if (!c) return HDG_E_ARG;
    if (!u || !lambda || !lam_bnd) return fail(c, HDG_E_ARG, "null pointer");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(c, HDG_E_ARG, "dt must be positive");
    if (scheme != HDG_BACKWARD_EULER && scheme != HDG_DIRK33) return fail(c, HDG_E_ARG, "unknown scheme");
    (void)t;
    double Dm[3][3];
    const int ns = step_tableau(scheme, Dm);
    const int64_t nl = c->n_local_dofs * c->nrhs;
    const int64_t nt = c->n_trace_dofs * c->nrhs;
    if (!c->d_stage) {
        int s = dalloc(c, &c->d_stage, 3 * nl);
        if (s) return s;
        if ((s = dalloc(c, &c->d_ustar, nl))) return s;
        if ((s = dalloc(c, &c->d_fstage, nl))) return s;
    }
    const double a = Dm[0][0] / dt;   // every stage of both schemes has this coefficient
    c->sg_replayed = false;
    hdg_ctx::StepKey key;
    key.dt = dt;
    key.scheme = scheme;
    key.u = u;
    key.lambda = lambda;
    key.lam_bnd = lam_bnd;
    key.src = src;
    int retry_nit = 0;   // > 0: the replay ran out of CG iterations; recapture with at least this many
    if (c->graph_step && c->sgexec && c->sg_key == key &&
        (!c->sg_reuse || (c->factors_cached && c->condensed && c->last_a == a))) {
        HIPCHK(hipGraphLaunch(c->sgexec, c->stream));
        // a graph that condenses assembles K again: copies derived from K are out of date
        if (!c->sg_reuse) ++c->mat_version;
        int h[8] = {}, st = 0;
        HIPCHK(hipMemcpyAsync(h, c->d_cgflags, 2 * ns * sizeof(int), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipMemcpyAsync(&st, c->d_status, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        if (st & 1) return fail(c, HDG_E_SINGULAR, "zero or non-finite pivot in a local factorisation");
        bool ok = true;
        for (int i = 0; i < ns; ++i) ok = ok && h[2 * i] == 1;
        if (ok) {
            HIPCHK(hipMemcpyAsync(u, c->d_stage + (ns - 1) * nl, nl * sizeof(double), hipMemcpyDeviceToDevice,
                                  c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
            c->last_iters = h[2 * (ns - 1) + 1];
            c->last_a = a;
            c->condensed = true;
            c->z_consumed = false;
            if (!c->sg_reuse) c->factors_cached = c->d_LU != nullptr && c->nrhs == 1;
            c->sg_replayed = true;
            return HDG_OK;
        }
        // a stage did not converge within the captured iterations (or went non-finite): u is
        // untouched, so the step runs again below without the graph, which reports a failure
        // properly, and the graph is captured again with a larger budget
        retry_nit = std::min(c->krylov_maxit, 2 * c->sg_nit);
    }
    int max_it = 0;
    for (int i = 0; i < ns; ++i) {
        int s = stage_rhs(c, i, Dm, dt, u, src);
        if (s) return fail(c, HDG_E_HIP, "stage right-hand-side launch failed");
        // the stage matrices depend on a only: with cached factors a repeated a needs only the
        // right-hand side condensed
        const bool reuse = c->cache_factors && c->factors_cached && c->condensed && a == c->last_a;
        s = reuse ? hdg_condense_rhs(c, a, c->d_fstage, lam_bnd + i * nt)
                  : hdg_condense(c, a, c->d_fstage, lam_bnd + i * nt);
        if (s) return s;
        int it;
        double rr;
        if ((s = hdg_trace_solve(c, lambda, &it, &rr))) return s;
        max_it = std::max(max_it, it);
        if ((s = hdg_recover(c, lambda, c->d_stage + i * nl))) return s;
    }
    // stiffly accurate: u^{n+1} = U_s
    HIPCHK(hipMemcpyAsync(u, c->d_stage + (ns - 1) * nl, nl * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (c->graph_step) {
        // capture for the next step with these arguments: the CG budget is the most iterations a
        // stage took here plus a margin (iterations past convergence return at once)
        const bool reuse = c->cache_factors && c->factors_cached && c->condensed && a == c->last_a;
        const int nit = std::min(c->krylov_maxit, std::max(retry_nit, max_it + max_it / 4 + 8));
        if (c->precond == HDG_PC_SSOR && ssor_supported(c) && c->nrhs == 1) {
            const int s = trace_ssor_alloc(c);   // no allocation inside the capture
            if (s) return fail(c, s, "allocation of the SSOR buffers failed");
        }
        if (capture_step(c, ns, Dm, dt, u, lambda, lam_bnd, src, reuse, nit))
            return fail(c, HDG_E_HIP, "capture of the step graph failed");
        c->sg_key = key;
    }
    return HDG_OK;
}

hdg_status hdg_volume_points(const hdg_ctx* c, double* pts) {
    if (!c || !pts) return HDG_E_ARG;
    if (c->vardeg) return HDG_E_UNSUPPORTED;
    std::vector<double> p, w;
    simplex_quadrature(c->dim, c->k + 2, p, w);
    const int d = c->dim, nq = (int)w.size();
    for (int64_t e = 0; e < c->n_elem; ++e) {
        const int64_t* ev = &c->ev[e * (d + 1)];
        for (int q = 0; q < nq; ++q)
            for (int r = 0; r < d; ++r) {
                double x = c->xyz[ev[0] * d + r];
                for (int s = 0; s < d; ++s) x += (c->xyz[ev[s + 1] * d + r] - c->xyz[ev[0] * d + r]) * p[q * d + s];
                pts[(e * nq + q) * d + r] = x;
            }
    }
    return HDG_OK;
}

hdg_status hdg_project_volume(const hdg_ctx* c, const double* vals, double* u) {
    if (!c || !vals || !u) return HDG_E_ARG;
    if (c->vardeg) return HDG_E_UNSUPPORTED;
    std::vector<double> p, w;
    simplex_quadrature(c->dim, c->k + 2, p, w);
    const int d = c->dim, nq = (int)w.size(), N = c->N, m = c->m_local;
    std::vector<double> phi(nq * N);
    for (int q = 0; q < nq; ++q) pkd_eval(d, c->k, &p[q * d], &phi[q * N], nullptr);
    for (int64_t e = 0; e < c->n_elem; ++e)
        for (int comp = 0; comp < m; ++comp)
            for (int i = 0; i < N; ++i) {
                double acc = 0.0;
                for (int q = 0; q < nq; ++q) acc += w[q] * phi[q * N + i] * vals[(e * nq + q) * m + comp];
                u[e * m * N + comp * N + i] = acc;
            }
    return HDG_OK;
}

hdg_status hdg_boundary_points(const hdg_ctx* c, double* pts) {
    if (!c || !pts) return HDG_E_ARG;
    if (c->vardeg) return HDG_E_UNSUPPORTED;
    std::vector<double> p, w;
    const int d = c->dim;
    simplex_quadrature(d - 1, c->k + 3, p, w);
    const int nq = (int)w.size();
    for (size_t b = 0; b < c->bface_list.size(); ++b) {
        const int64_t* fv = &c->face_vert[c->bface_list[b] * d];
        for (int q = 0; q < nq; ++q)
            for (int r = 0; r < d; ++r) {
                double x = c->xyz[fv[0] * d + r];
                for (int s = 0; s < d - 1; ++s)
                    x += (c->xyz[fv[s + 1] * d + r] - c->xyz[fv[0] * d + r]) * p[q * (d - 1) + s];
                pts[(b * nq + q) * d + r] = x;
            }
    }
    return HDG_OK;
}

hdg_status hdg_project_boundary(const hdg_ctx* c, const double* vals, double* lam) {
    if (!c || !vals || !lam) return HDG_E_ARG;
    if (c->vardeg) return HDG_E_UNSUPPORTED;
    std::vector<double> p, w;
    const int d = c->dim;
    simplex_quadrature(d - 1, c->k + 3, p, w);
    const int nq = (int)w.size(), NF = c->NF, mt = c->m_trace;
    std::vector<double> psi(nq * NF);
    for (int q = 0; q < nq; ++q) pkd_eval(d - 1, c->k, &p[q * (d - 1)], &psi[q * NF], nullptr);
    std::fill(lam, lam + c->n_trace_dofs, 0.0);
    const int vw = (c->physics == HDG_ACOUSTIC) ? 1 : 3;
    for (size_t b = 0; b < c->bface_list.size(); ++b) {
        int64_t F = c->bface_list[b];
        // Dirichlet: the projection (face mass = s_F I, the quadrature sum carries s_F);
        // Neumann: the tested datum <g, psi_l>_F = s_F times that sum
        double sF = 1.0;
        if (c->face_bnd[F] == 2) {
            const int64_t* fv = &c->face_vert[F * d];
            double T[2][3] = {};
            for (int s2 = 0; s2 + 1 < d; ++s2)
                for (int r = 0; r < d; ++r) T[s2][r] = c->xyz[fv[s2 + 1] * d + r] - c->xyz[fv[0] * d + r];
            if (d == 3) {
                const double cx = T[0][1] * T[1][2] - T[0][2] * T[1][1];
                const double cy = T[0][2] * T[1][0] - T[0][0] * T[1][2];
                const double cz = T[0][0] * T[1][1] - T[0][1] * T[1][0];
                sF = std::sqrt(cx * cx + cy * cy + cz * cz);
            } else {
                sF = std::sqrt(T[0][0] * T[0][0] + T[0][1] * T[0][1]);
            }
        }
        for (int comp = 0; comp < mt; ++comp)
            for (int l = 0; l < NF; ++l) {
                double acc = 0.0;
                for (int q = 0; q < nq; ++q) {
                    const double* v = &vals[(b * nq + q) * vw];
                    double g;
                    if (c->physics == HDG_MAXWELL || c->physics == HDG_MAXWELL_GLM) {
                        const double* t = &c->frame[F * 6 + comp * 3];
                        g = v[0] * t[0] + v[1] * t[1] + v[2] * t[2];
                    } else {
                        g = v[comp];
                    }
                    acc += w[q] * psi[q * NF + l] * g;
                }
                lam[F * c->bs + comp * NF + l] = sF * acc;
            }
    }
    return HDG_OK;
}

hdg_status hdg_point_sources(const hdg_ctx* c, int n_src, const double* pts, double* f) {
    if (!c || !pts || !f || n_src < 1) return HDG_E_ARG;
    if (c->physics != HDG_ACOUSTIC) return HDG_E_UNSUPPORTED;
    const int d = c->dim;
    std::fill(f, f + c->n_local_dofs * n_src, 0.0);
    std::vector<double> phi(c->N);
    for (int s = 0; s < n_src; ++s) {
        const double* x = pts + s * d;
        bool found = false;
        for (int64_t e = 0; e < c->n_elem && !found; ++e) {
            const double* g = &c->geom[e * GEOM_STRIDE];
            const int64_t v0 = c->ev[e * (d + 1)];
            double xi[3], sum = 0.0;
            bool inside = true;
            for (int r = 0; r < d; ++r) {
                double acc = 0.0;
                for (int xx = 0; xx < d; ++xx) acc += g[1 + r * d + xx] * (x[xx] - c->xyz[v0 * d + xx]);
                xi[r] = acc;
                sum += acc;
                if (acc < -1e-12) inside = false;
            }
            if (!inside || sum > 1.0 + 1e-12) continue;
            const int ke = c->vardeg ? c->degree[e] : c->k, Ne = dim_p(ke, d);
            const int64_t base = c->vardeg ? c->loc_off_h[e] : e * c->n_loc;
            pkd_eval(d, ke, xi, phi.data(), nullptr);
            for (int i = 0; i < Ne; ++i) f[(base + d * Ne + i) * n_src + s] = phi[i];
            found = true;
        }
        if (!found) return HDG_E_ARG;
    }
    return HDG_OK;
}

hdg_status hdg_element_data(hdg_ctx* c, int which, int64_t e0, int64_t count, double* out) {
    if (!c || !out || which < 0 || which > 3 || e0 < 0 || count < 0 || e0 + count > c->n_elem) return HDG_E_ARG;
    if (!c->condensed) return fail(c, HDG_E_STATE, "no condensed data");
    if (c->vardeg && which == 3) return fail(c, HDG_E_UNSUPPORTED, "z rows are per-class on variable degree");
    const int64_t R = c->nrhs, n = c->n_loc, t = c->n_tr;
    int64_t blk;
    void* src;
    const int64_t ns = c->Ns;
    switch (which) {
        case 0: blk = t * t; src = c->d_Ke; break;
        case 1: blk = t * R; src = c->d_re; break;
        case 2: blk = ns * t; src = c->d_Zt; break;
        default: blk = n * R; src = c->d_z; break;
    }
    const size_t tsz = (c->precision == HDG_FP64) ? sizeof(double) : sizeof(float);
    std::vector<char> buf(count * blk * tsz);
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(buf.data(), (char*)src + e0 * blk * tsz, buf.size(), hipMemcpyDeviceToHost));
    const int64_t oblk = (which == 3) ? ns * R : blk;
    for (int64_t e = 0; e < count; ++e)
        for (int64_t i = 0; i < oblk; ++i) {
            // which == 3: only the Schur-block rows of z are A^{-1} f (the eliminated rows hold
            // the closed-form part applied at recovery)
            int64_t src_i = (which == 3) ? c->s_row0 * R + i : i;
            if (which == 2 && c->fast_ac) src_i = (i % t) * ns + i / t;   // Z_p stored column-major
            if (which == 0 && c->ke_tile > 0) {   // K_e stored by its upper tiles
                const int64_t r = i / t, cc = i % t;
                if (r / c->ke_tile > cc / c->ke_tile) src_i = cc * t + r;
            }
            int64_t k = e * blk + src_i;
            out[e * oblk + i] = (tsz == 8) ? ((double*)buf.data())[k] : (double)((float*)buf.data())[k];
        }
    return HDG_OK;
}

hdg_status hdg_last_timing(const hdg_ctx* c, int which, double* ms) {
    if (!c || !ms) return HDG_E_ARG;
    const float v[6] = {c->tim.condense, c->tim.assemble, c->tim.solve, c->tim.recover, c->tim.refine_elem,
                        c->tim.refine_solve};
    if (which < 0 || which > 5) return HDG_E_ARG;
    *ms = v[which];
    return HDG_OK;
}

void hdg_destroy(hdg_ctx* c) {
    if (!c) return;
    void* ptrs[] = {c->d_geom, c->d_eface, c->d_eperm, c->d_face_elem, c->d_face_lf, c->d_face_bnd,
                    c->d_bsr_cols, c->tab.Sr, c->tab.Mf, c->tab.Tsym, c->tab.Ef, c->tab.Sr32, c->tab.Mf32,
                    c->tab.Tsym32, c->tab.Ef32, c->tab.Tfull, c->tab.Tfull32, c->tab.SrT, c->tab.EfT, c->d_eframe, c->d_xscratch, c->d_Ke, c->d_re, c->d_Zt, c->d_z, c->d_LU, c->d_status,
                    c->d_bsr, c->d_bsr32, c->d_rhs, c->d_pinv, c->d_cg_r, c->d_cg_z, c->d_cg_p, c->d_cg_q, c->d_red,
                    c->d_scal, c->d_f_saved, c->d_lbnd_saved, c->d_su, c->d_slam, c->d_du, c->d_dlam,
                    c->d_re64, c->d_sq, c->d_cgflags, c->d_cfaces, c->d_ssoff, c->d_ssnb, c->d_ssdst, c->d_ss, c->d_ssA, c->d_rinv,
                    c->d_stage, c->d_ustar, c->d_fstage, c->d_loc_off, c->d_efnf, c->d_face_nf, c->d_edeg,
                    c->d_cls[1], c->d_cls[2], c->d_cls[3], c->d_cls[4], c->d_cls[5]};
    if (c->stream || c->d_geom) (void)hipStreamSynchronize(c->stream);
    for (void* p : ptrs) dfree(c, p);
    for (auto& t : c->tabk) {
        void* tp[] = {t.Sr, t.Mf, t.Tsym, t.Ef, t.Tfull, t.Sr32, t.Mf32, t.Tsym32, t.Ef32, t.Tfull32, t.SrT, t.EfT};
        for (void* p : tp) dfree(c, p);
    }
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->ev_rr) (void)hipEventDestroy(c->ev_rr);
    if (c->h_rr) (void)hipHostFree(c->h_rr);
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->sgexec) (void)hipGraphExecDestroy(c->sgexec);
    if (c->sg_stream) (void)hipStreamDestroy(c->sg_stream);
    for (int i = 0; i < 6; ++i) {
        if (c->side[i]) {
            (void)hipStreamSynchronize(c->side[i]);
            (void)hipStreamDestroy(c->side[i]);
        }
        if (c->ev_join[i]) (void)hipEventDestroy(c->ev_join[i]);
    }
    hipEvent_t evs[] = {c->ev_fork, c->ev_in, c->ev_out};
    for (hipEvent_t e : evs)
        if (e) (void)hipEventDestroy(e);
    delete c;
}

// Host-only access to the reference tables (no device needed): which = 0 Sr, 1 Mf, 2 Tsym,
// 3 oriented face table E (face degree kF).  Returns the number of doubles written, or a
// negative hdg_status.
int64_t hdg_reference_table(int dim, int k, int kF, int which, double* out, int64_t cap) {
    if ((dim != 2 && dim != 3) || k < 0 || k > 8 || kF < 0 || kF > 8 || !out) return -HDG_E_ARG;
    std::vector<double> v;
    if (which <= 2) {
        RefTables T;
        build_ref_tables(dim, k, T);
        v = (which == 0) ? T.Sr : (which == 1 ? T.Mf : T.Tsym);
    } else if (which == 3) {
        RefFaceTables E;
        build_face_tables(dim, k, kF, E);
        v = E.E;
    } else {
        return -HDG_E_ARG;
    }
    if ((int64_t)v.size() > cap) return -HDG_E_ARG;
    std::copy(v.begin(), v.end(), out);
    return (int64_t)v.size();
}

}  // extern "C"
