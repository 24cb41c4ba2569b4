// Stage glue (section 2.3.2): f = a Mw u element by element.  With the orthonormal basis the
// weight matrix of each element is |J| times a small matrix over field components:
//   acoustic  diag(rho, .., rho, 1/(rho c^2))
//   elastic   compliance Acomp on the six stress components (off-diagonal test tensors
//             weigh twice), rho on the velocity
//   maxwell   diag(mu, mu, mu, eps, eps, eps)
//   maxwell with the GLM multiplier: the same and 1/alpha_1^2 = 1 on phi
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.h"

namespace hdg {

namespace {
constexpr int NT = 256;

__global__ __launch_bounds__(NT) void apply_mass_kernel(int64_t ne, int physics, int m, int N, int R, double a,
                                                        const double* __restrict__ geom,
                                                        const double* __restrict__ u, double* __restrict__ f) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)m * N * R;
    if (gid >= ne * per) return;
    int64_t e = gid / per;
    int rem = (int)(gid % per);
    int comp = rem / (N * R);
    int iq = rem % (N * R);
    const double* g = geom + e * GEOM_STRIDE;
    const double J = g[0];
    const double* par = g + GEO_PAR;
    const double* ue = u + e * per;
    double w;
    if (physics == HDG_ACOUSTIC) {
        w = (comp < m - 1) ? par[0] : 1.0 / (par[0] * par[1] * par[1]);
        f[gid] = a * J * w * ue[rem];
        return;
    }
    if (physics == HDG_MAXWELL || physics == HDG_MAXWELL_GLM) {
        // GLM: the multiplier's weight is 1 / alpha_1^2 = 1 (section 5.4)
        w = (comp < 3) ? par[1] : (comp < 6 ? par[0] : 1.0);
        f[gid] = a * J * w * ue[rem];
        return;
    }
    // elastic
    if (comp >= 6) {
        f[gid] = a * J * par[0] * ue[rem];
        return;
    }
    const double lam = par[1], mu = par[2];
    const double c0 = lam / (3.0 * lam + 2.0 * mu);
    double acc;
    if (comp < 3) {
        double tr = ue[0 * N * R + iq] + ue[1 * N * R + iq] + ue[2 * N * R + iq];
        acc = (ue[comp * N * R + iq] - c0 * tr) / (2.0 * mu);
    } else {
        acc = 2.0 * ue[comp * N * R + iq] / (2.0 * mu);
    }
    f[gid] = a * J * acc;
}
// acoustics on a mesh of variable degree: one workgroup per element, compact local layout
__global__ __launch_bounds__(NT) void apply_mass_var_kernel(int64_t ne, int m, int R, double a,
                                                            const double* __restrict__ geom,
                                                            const int64_t* __restrict__ loc_off,
                                                            const double* __restrict__ u, double* __restrict__ f) {
    for (int64_t e = blockIdx.x; e < ne; e += gridDim.x) {
        const double* g = geom + e * GEOM_STRIDE;
        const double J = g[0];
        const double* par = g + GEO_PAR;
        const int64_t b0 = loc_off[e] * R, n = (loc_off[e + 1] - loc_off[e]) * R;
        const int64_t Nr = n / m;   // basis functions x rhs per component
        for (int64_t i = threadIdx.x; i < n; i += NT) {
            const int comp = (int)(i / Nr);
            const double w = (comp < m - 1) ? par[0] : 1.0 / (par[0] * par[1] * par[1]);
            f[b0 + i] = a * J * w * u[b0 + i];
        }
    }
}
}  // namespace

int launch_apply_mass(hdg_ctx* c, double a, const double* u, double* f) {
    if (c->vardeg) {
        const int grid = (int)std::min<int64_t>(c->n_elem, 65536);
        hipLaunchKernelGGL(apply_mass_var_kernel, dim3(grid), dim3(NT), 0, c->stream, c->n_elem, c->m_local, c->nrhs,
                           a, c->d_geom, c->d_loc_off, u, f);
        return (int)hipGetLastError();
    }
    int64_t n = c->n_elem * (int64_t)c->n_loc * c->nrhs;
    hipLaunchKernelGGL(apply_mass_kernel, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, c->stream, c->n_elem,
                       c->physics, c->m_local, c->N, c->nrhs, a, c->d_geom, u, f);
    return (int)hipGetLastError();
}

}  // namespace hdg
